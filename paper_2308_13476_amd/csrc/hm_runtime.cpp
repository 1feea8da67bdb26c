// Host runtime of the multigrid solver: workspace layout, hierarchy setup,
// cycle scheduling and the C ABI declared in include/helmg.h.
#include "helmg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <complex>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hm_kernels.hpp"

using namespace hm;

namespace {

thread_local std::string g_setup_error;

// Device scratch of mg_residual_noalloc: a file-scope array that every GPU the
// library runs on holds until the process ends. Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device (with that device current), and is
// kept in g_scratch_ptr.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The scratch address on the current device, looked up on the first call per
// device.
hipError_t static_scratch(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

constexpr size_t kAlign = 256;
constexpr int kMaxCoarseNodes = 1089;
constexpr int kMaxN = 4096;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

Grid make_grid(int n) {
    Grid g;
    g.n = n;
    const int m = n + 1;
    g.pitch = int(align_up(size_t(kGhostX + m + kGhost), kPitchAlign));
    g.plane = (long long)align_up(size_t(g.pitch) * size_t(m + 2 * kGhost), 64);
    return g;
}

int next_radius(int r, int transfer) { return transfer == MG_TRANSFER_BEZIER ? (r + 4) / 2 : (r + 2) / 2; }

struct LevelBuf {
    Grid g;
    int radius = 1;
    cplx<double>* coef64 = nullptr;
    cplx<float>* coef32 = nullptr;
    // [max_batch] planes each; V holds 4 planes per right-hand side
    cplx<double>* u64 = nullptr; cplx<double>* f64 = nullptr; cplx<double>* t64 = nullptr;
    cplx<double>* w64 = nullptr; cplx<double>* V64 = nullptr;
    cplx<float>* u32 = nullptr; cplx<float>* f32 = nullptr; cplx<float>* t32 = nullptr;
    cplx<float>* w32 = nullptr; cplx<float>* V32 = nullptr;
};

// Sequential carve of the caller's workspace (base == nullptr only measures).
struct Carver {
    char* base;
    size_t off = 0;
    template <typename P>
    P* take(size_t bytes) {
        off = align_up(off, kAlign);
        P* p = base ? reinterpret_cast<P*>(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

}  // namespace

struct mg_ctx {
    int n = 0, L = 0, transfer = 0, max_batch = 1, has32 = 0, coarsest_n = 4;
    int device = -1;  // HIP device current at mg_setup (the workspace's device)
    double h = 0.0, shift = 0.0;
    std::vector<LevelBuf> lv;
    double* k2_64 = nullptr;
    float* k2_32 = nullptr;
    cplx<double>* dense = nullptr;
    int* piv = nullptr;
    cplx<double>* inv = nullptr;  // explicit coarsest inverse (small coarsest grids only)
    GmState* gm = nullptr;
    RhsNorms* norms = nullptr;
    int* active = nullptr;
    int* stop_count = nullptr;      // [max_batch] stop tests taken per right-hand side
    double* stop_limits = nullptr;  // [max_batch][2] tolerance, divergence limit
    double* partials = nullptr;
    int* k2_flags = nullptr;  // [2] result of the k^2 check
    char* ws = nullptr;
    size_t ws_bytes = 0;
    // host mirrors (pinned)
    RhsNorms* h_norms = nullptr;
    int* h_active = nullptr;
    double* h_limits = nullptr;
    RhsReport* h_ring = nullptr;  // stop-test reports, written by the device
    hipEvent_t cycle_done[2] = {nullptr, nullptr};
    // FGMRES: two slots of Hessenberg columns read back while the next
    // iteration runs (allocated by the first FGMRES solve), and their events
    cplx<double>* h_hcol = nullptr;
    hipEvent_t hcol_done[2] = {nullptr, nullptr};
    std::string err;
    // kernel timing hook: event pairs of eager launches, and of the graph run last
    int timing_class = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    int t_launches = 0;
    double t_ms = 0.0, t_nodes = 0.0;
    // captured cycles (one per configuration and buffer assignment)
    struct GraphEntry {
        std::vector<uintptr_t> key;
        hipGraphExec_t exec = nullptr;
        std::vector<std::pair<hipEvent_t, hipEvent_t>> timed;
        double timed_nodes = 0.0;
        std::vector<void*> after_ptrs;
        int after_cur = 0;
        std::vector<int> marks;  // graph_marks left by the captured body
    };
    std::vector<GraphEntry> graphs;
    // host bookkeeping that a cycle body records while it enqueues (the
    // buffer parity after each of its cycles); replays restore it
    std::vector<int> graph_marks;
    int last_graph = -1;
    hipStream_t cap_stream = nullptr;
    bool use_graph = true;
    // first level run by the single-workgroup coarse tail (-1: none), per
    // precision (index 0: FP64 cycles, 1: FP32 cycles), for tail levels of at
    // most tail_n intervals
    int tail_level[2] = {-1, -1};
    int tail_n = 16;
    // level 1 applied as R C_s P from level-0 data instead of its stored
    // stencil: 1 in FP32 cycles, 2 in both, 0 never (default: the stored
    // stencil, read as its upper half, is faster in both precisions)
    // (HELMG_L1_PRODUCT)
    int product_l1 = 0;
    // blocks per right-hand side that a level grid aims at (HELMG_MAX_BLOCKS;
    // max(64, 640 / max_batch) on batch handles); beyond it reductions are
    // pre-reduced in a one-block pass
    int block_cap = 640;
    // block heights: light kernels on grids of >= 256 intervals (4, 8, 16;
    // HELMG_TALL_BLOCKS) and every kernel on grids of <= 128 intervals (2 or 4;
    // HELMG_SMALL_ROWS)
    int tall_rows = 4, small_rows = 2;
    // JSON file of autotuned launch settings (mg_setup_opts.tune_cache), or empty
    std::string tune_cache;
    // the coarse grid correction folded into the first post-smoothing pass
    // where its LDS stage fits (HELMG_FUSE_CORRECTION=0: always a pass of its own)
    int fuse_correction = 1;
    // the restriction folded into the last pre-smoothing pass of GMRES cycles
    // (HELMG_FUSE_RESTRICT=0: always a pass of its own)
    int fuse_restrict = 1;
    // on level 0 of FP32 cycles the first apply pass of the post-smoothing
    // step is folded into the correction pass before it (HELMG_FUSE_R_A0=0:
    // a pass of its own)
    int fuse_r_a0 = 1;
    // HELMG_LOG=1: one line per right-hand side and cycle on stderr (relative
    // residual, contraction, stop decision) as the host reads the reports
    int log = 0;
    // weighted-Jacobi sweeps two per pass where the level allows it
    // (HELMG_JACOBI_PAIRS=0: one per pass)
    int jacobi_pairs = 1;
    // the update pass of a coarse level's last post-smoothing GMRES step is
    // formed by the next finer level's correction pass instead of launched
    // (HELMG_DEFER_UPDATE=0: always launched)
    int defer_update = 1;
    // which of u64 / t64 holds the level-0 FP64 iterate of each right-hand side
    int cur_buf = 0;
    std::vector<int> final_buf;
};

namespace {

// ---------------------------------------------------------------- layout plan
bool levels_for(int n, int levels, int coarsest_n, int* L_out, std::string* why) {
    if (n < 2) { *why = "n must be >= 2"; return false; }
    // level kernels launch at most kMaxPartialBlocks blocks per right-hand side
    if (n > kMaxN) { *why = "n must be <= 4096"; return false; }
    int L = levels;
    if (L <= 0) {
        if (coarsest_n < 1) { *why = "coarsest_n must be >= 1"; return false; }
        L = 1;
        int m = n;
        while (m > coarsest_n) {
            if (m % 2) { *why = "n cannot be halved down to coarsest_n"; return false; }
            m /= 2;
            ++L;
        }
        if (m != coarsest_n) { *why = "n is not coarsest_n times a power of two"; return false; }
    }
    if (L < 2) { *why = "need at least two levels"; return false; }
    if (L > 24 || n % (1 << (L - 1)) != 0) { *why = "n must be divisible by 2^(levels-1)"; return false; }
    const int nc = n >> (L - 1);
    if ((nc + 1) * (nc + 1) > kMaxCoarseNodes) { *why = "coarsest grid larger than 32 x 32 intervals"; return false; }
    *L_out = L;
    return true;
}

size_t carve(mg_ctx* c, char* base, int n, int L, int transfer, int max_batch, int has32) {
    Carver cv{base};
    if (c) c->lv.assign(L, LevelBuf());
    int r = 1;
    const size_t B = size_t(max_batch);
    for (int l = 0; l < L; ++l) {
        const Grid g = make_grid(n >> l);
        LevelBuf tmp;
        LevelBuf& lb = c ? c->lv[l] : tmp;
        lb.g = g;
        lb.radius = (l == 0) ? 1 : r;
        const size_t pl = size_t(g.plane);
        const size_t ncoef = size_t(2 * lb.radius + 1) * size_t(2 * lb.radius + 1);
        if (l > 0) {
            lb.coef64 = cv.take<cplx<double>>(ncoef * pl * 16);
            if (has32) lb.coef32 = cv.take<cplx<float>>(ncoef * pl * 8);
        }
        lb.u64 = cv.take<cplx<double>>(B * pl * 16);
        lb.f64 = cv.take<cplx<double>>(B * pl * 16);
        lb.t64 = cv.take<cplx<double>>(B * pl * 16);
        lb.w64 = cv.take<cplx<double>>(B * pl * 16);
        lb.V64 = cv.take<cplx<double>>(4 * B * pl * 16);
        if (has32) {
            lb.u32 = cv.take<cplx<float>>(B * pl * 8);
            lb.f32 = cv.take<cplx<float>>(B * pl * 8);
            lb.t32 = cv.take<cplx<float>>(B * pl * 8);
            lb.w32 = cv.take<cplx<float>>(B * pl * 8);
            lb.V32 = cv.take<cplx<float>>(4 * B * pl * 8);
        }
        r = next_radius(lb.radius, transfer);
    }
    const Grid g0 = make_grid(n);
    double* k64 = cv.take<double>(size_t(g0.plane) * 8);
    float* k32 = has32 ? cv.take<float>(size_t(g0.plane) * 4) : nullptr;
    const int nc = n >> (L - 1);
    const size_t Nc = size_t(nc + 1) * size_t(nc + 1);
    cplx<double>* dense = cv.take<cplx<double>>(Nc * Nc * 16);
    int* piv = cv.take<int>(Nc * 4);
    cplx<double>* inv = Nc <= size_t(kTailMaxCoarseNodes) ? cv.take<cplx<double>>(Nc * Nc * 16) : nullptr;
    GmState* gm = cv.take<GmState>(B * sizeof(GmState));
    RhsNorms* norms = cv.take<RhsNorms>(B * sizeof(RhsNorms));
    int* active = cv.take<int>(B * 4);
    int* stop_count = cv.take<int>(B * 4);
    double* stop_limits = cv.take<double>(B * 16);
    double* partials = cv.take<double>(2 * B * size_t(kPartStride) * 8);
    int* k2_flags = cv.take<int>(2 * 4);
    if (c) {
        c->k2_flags = k2_flags;
        c->k2_64 = k64;
        c->k2_32 = k32;
        c->dense = dense;
        c->piv = piv;
        c->inv = inv;
        c->gm = gm;
        c->norms = norms;
        c->active = active;
        c->stop_count = stop_count;
        c->stop_limits = stop_limits;
        c->partials = partials;
    }
    return align_up(cv.off, kAlign);
}

// ---------------------------------------------------------------- helpers
#define HM_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            c->err = std::string(#call) + ": " + hipGetErrorString(e_);                 \
            return MG_E_HIP;                                                             \
        }                                                                                \
    } while (0)

mg_status check_launch(mg_ctx* c) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->err = std::string("kernel launch: ") + hipGetErrorString(e);
        return MG_E_HIP;
    }
    return MG_OK;
}

template <typename T> struct Prec;
template <> struct Prec<double> {
    static cplx<double>* u(LevelBuf& l) { return l.u64; }
    static cplx<double>*& u_ref(LevelBuf& l) { return l.u64; }
    static cplx<double>* f(LevelBuf& l) { return l.f64; }
    static cplx<double>*& t_ref(LevelBuf& l) { return l.t64; }
    static cplx<double>* w(LevelBuf& l) { return l.w64; }
    static cplx<double>* V(LevelBuf& l) { return l.V64; }
    static const cplx<double>* coef(const LevelBuf& l) { return l.coef64; }
    static const double* k2(const mg_ctx* c) { return c->k2_64; }
    static constexpr double breakdown = 1e-14;
};
template <> struct Prec<float> {
    static cplx<float>* u(LevelBuf& l) { return l.u32; }
    static cplx<float>*& u_ref(LevelBuf& l) { return l.u32; }
    static cplx<float>* f(LevelBuf& l) { return l.f32; }
    static cplx<float>*& t_ref(LevelBuf& l) { return l.t32; }
    static cplx<float>* w(LevelBuf& l) { return l.w32; }
    static cplx<float>* V(LevelBuf& l) { return l.V32; }
    static const cplx<float>* coef(const LevelBuf& l) { return l.coef32; }
    static const float* k2(const mg_ctx* c) { return c->k2_32; }
    static constexpr double breakdown = 1e-6;
};

template <typename T>
LevelOp<T> level_op(const mg_ctx* c, int l) {
    const LevelBuf& lb = c->lv[l];
    const int product = c->product_l1 == 2 || (c->product_l1 == 1 && sizeof(T) == 4);
    return LevelOp<T>{l, lb.g, lb.radius, Prec<T>::coef(lb), Prec<T>::k2(c), c->h,
                      product, c->lv[0].g, c->shift, c->transfer};
}

template <typename T>
Vec<T> vec(cplx<T>* p, const LevelBuf& lb) { return Vec<T>{p, lb.g.plane}; }

LaunchCtx launch_ctx(mg_ctx* c, hipStream_t s, int nrhs) {
    LaunchCtx lc{s, nrhs, c->active, c->partials, c->max_batch, c->block_cap, c->fuse_correction};
    lc.fuse_restrict = c->fuse_restrict;
    lc.fuse_r_a0 = c->fuse_r_a0;
    lc.tall_rows = c->tall_rows;
    lc.small_rows = c->small_rows;
    return lc;
}

// Timing hook: events around the launches of one kernel class.
struct TimedScope {
    mg_ctx* c;
    hipStream_t s;
    bool on;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double nodes;
    TimedScope(mg_ctx* c_, hipStream_t s_, int cls, double nodes_)
        : c(c_), s(s_), on(c_->timing_class == cls && cls > 0), nodes(nodes_) {
        if (!on) return;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            on = false;
            return;
        }
        (void)hipEventRecord(e0, s);
    }
    ~TimedScope() {
        if (!on) return;
        (void)hipEventRecord(e1, s);
        c->ev_pending.push_back({e0, e1});
        c->t_nodes += nodes;
    }
};

void harvest_pairs(mg_ctx* c, const std::vector<std::pair<hipEvent_t, hipEvent_t>>& pairs) {
    for (auto& pr : pairs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
            c->t_ms += ms;
            c->t_launches += 1;
        }
    }
}

void destroy_pairs(std::vector<std::pair<hipEvent_t, hipEvent_t>>& pairs) {
    for (auto& pr : pairs) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    pairs.clear();
}

// Called after the stream has been synchronised.
void harvest_timing(mg_ctx* c) {
    harvest_pairs(c, c->ev_pending);
    destroy_pairs(c->ev_pending);
    if (c->last_graph >= 0) {
        const auto& e = c->graphs[c->last_graph];
        harvest_pairs(c, e.timed);
        c->t_nodes += e.timed_nodes;
        c->last_graph = -1;
    }
}

std::vector<void*> pointer_state(const mg_ctx* c) {
    std::vector<void*> v;
    for (const LevelBuf& l : c->lv) {
        v.push_back(l.u64);
        v.push_back(l.t64);
        v.push_back(l.u32);
        v.push_back(l.t32);
    }
    return v;
}

void restore_pointer_state(mg_ctx* c, const std::vector<void*>& v) {
    size_t q = 0;
    for (LevelBuf& l : c->lv) {
        l.u64 = static_cast<cplx<double>*>(v[q++]);
        l.t64 = static_cast<cplx<double>*>(v[q++]);
        l.u32 = static_cast<cplx<float>*>(v[q++]);
        l.t32 = static_cast<cplx<float>*>(v[q++]);
    }
}

// Runs body(stream) once: eagerly, or as a captured graph cached under `params`
// plus the current buffer assignment. The host-side buffer bookkeeping that the
// body performs is replayed from the cache on later launches.
template <typename F>
mg_status run_cycle_graph(mg_ctx* c, hipStream_t s, std::vector<uintptr_t> key, F&& body) {
    // per-kernel event timing needs eager launches (events recorded inside a
    // capture cannot be queried for elapsed time)
    if (!c->use_graph || c->timing_class != 0) {
        c->graph_marks.clear();
        body(s);
        return check_launch(c);
    }
    const std::vector<void*> before = pointer_state(c);
    for (void* p : before) key.push_back(reinterpret_cast<uintptr_t>(p));
    key.push_back(uintptr_t(c->cur_buf));
    for (size_t i = 0; i < c->graphs.size(); ++i) {
        if (c->graphs[i].key != key) continue;
        restore_pointer_state(c, c->graphs[i].after_ptrs);
        c->cur_buf = c->graphs[i].after_cur;
        c->graph_marks = c->graphs[i].marks;
        HM_HIP(hipGraphLaunch(c->graphs[i].exec, s));
        c->last_graph = int(i);
        return MG_OK;
    }
    if (!c->cap_stream) HM_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const int cur_before = c->cur_buf;
    const double nodes_before = c->t_nodes;
    destroy_pairs(c->ev_pending);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    c->graph_marks.clear();
    bool ok = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed) == hipSuccess;
    if (ok) {
        body(c->cap_stream);
        ok = hipStreamEndCapture(c->cap_stream, &graph) == hipSuccess && graph != nullptr;
    }
    if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (!ok) {
        // fall back to eager launches for the rest of this handle's life
        c->use_graph = false;
        destroy_pairs(c->ev_pending);
        c->t_nodes = nodes_before;
        restore_pointer_state(c, before);
        c->cur_buf = cur_before;
        c->graph_marks.clear();
        body(s);
        return check_launch(c);
    }
    mg_ctx::GraphEntry e;
    e.key = std::move(key);
    e.exec = exec;
    e.timed = std::move(c->ev_pending);
    c->ev_pending.clear();
    e.timed_nodes = c->t_nodes - nodes_before;
    c->t_nodes = nodes_before;
    e.after_ptrs = pointer_state(c);
    e.after_cur = c->cur_buf;
    e.marks = c->graph_marks;
    c->graphs.push_back(std::move(e));
    HM_HIP(hipGraphLaunch(c->graphs.back().exec, s));
    c->last_graph = int(c->graphs.size() - 1);
    return MG_OK;
}

// ---------------------------------------------------------------- cycle
// Drops every captured cycle (after a change of launch settings).
void clear_graphs(mg_ctx* c) {
    for (auto& g : c->graphs) {
        destroy_pairs(g.timed);
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    }
    c->graphs.clear();
    c->last_graph = -1;
}

struct CycleParams {
    int gamma, smoother, nu1, nu2;
    double omega;
};

// One smoothing step on level l. With then_residual (GMRES only), the step's
// last pass also forms the residual f - A u of the updated iterate into the
// level's w buffer. u_zero (GMRES): the step starts from u = 0, which u does
// not hold. defer (GMRES; may be null): the step's update pass is left to the
// caller, as launch_gmres_step describes.
template <typename T>
void smooth(mg_ctx* c, const LaunchCtx& lc, int l, const CycleParams& cp, bool then_residual = false,
            int r_ready_nblk = 0, ProlongIn<T> pro = ProlongIn<T>{}, bool u_zero = false,
            RestrictOut<T>* rout = nullptr, int jsteps = 1, DeferredUpdate<T>* defer = nullptr,
            bool w_ready = false) {
    LevelBuf& lb = c->lv[l];
    const LevelOp<T> op = level_op<T>(c, l);
    const double nodes = double(lb.g.n + 1) * (lb.g.n + 1) * lc.nrhs;
    if (cp.smoother == MG_JACOBI) {
        // jsteps = 2: two sweeps, in one pass where the level allows it
        if (pro.e.p) launch_prolong_add<T>(lc, pro.gc, lb.g, pro.transfer, pro.e, vec<T>(Prec<T>::u(lb), lb));
        auto swap_buffers = [&] {
            std::swap(Prec<T>::u_ref(lb), Prec<T>::t_ref(lb));
            if (l == 0 && sizeof(T) == 8) c->cur_buf ^= 1;
        };
        TimedScope ts(c, lc.stream, l == 0 ? 2 : -1, nodes * jsteps);
        if (jsteps == 2 && c->jacobi_pairs &&
            launch_jacobi2<T>(lc, op, vec<T>(Prec<T>::u(lb), lb), vec<T>(Prec<T>::f(lb), lb),
                              vec<T>(Prec<T>::t_ref(lb), lb), 1.0 / cp.omega)) {
            swap_buffers();
            return;
        }
        for (int k = 0; k < jsteps; ++k) {
            launch_jacobi<T>(lc, op, vec<T>(Prec<T>::u(lb), lb), vec<T>(Prec<T>::f(lb), lb),
                             vec<T>(Prec<T>::t_ref(lb), lb), 1.0 / cp.omega);
            swap_buffers();
        }
        return;
    }
    // timing hook: the second fused orthogonalise + apply pass (launch 3 of
    // the step) records a start and a stop event with its own dispatch
    const bool timed = c->timing_class == (l == 0 ? 1 : (l == 1 ? 4 : -1));
    hipEvent_t tev[2] = {nullptr, nullptr};
    if (timed && (hipEventCreate(&tev[0]) != hipSuccess || hipEventCreate(&tev[1]) != hipSuccess)) {
        if (tev[0]) (void)hipEventDestroy(tev[0]);
        tev[0] = tev[1] = nullptr;
    }
    const Vec<T> w = vec<T>(Prec<T>::w(lb), lb), t = vec<T>(Prec<T>::t_ref(lb), lb);
    launch_gmres_step<T>(lc, op, vec<T>(Prec<T>::u(lb), lb), vec<T>(Prec<T>::f(lb), lb), vec<T>(Prec<T>::V(lb), lb),
                         w, t, c->gm, Prec<T>::breakdown, tev[1] ? tev : nullptr,
                         then_residual ? w : Vec<T>{nullptr, 0}, r_ready_nblk, pro, u_zero, rout, defer, w_ready);
    if (tev[1]) {
        c->ev_pending.push_back({tev[0], tev[1]});
        c->t_nodes += nodes;
    }
}

template <typename T>
void launch_tail_from(mg_ctx* c, const LaunchCtx& lc, int l0, const CycleParams& cp, bool top_zero) {
    TailArgs<T> a{};
    a.nlev = c->L - l0;
    a.plane_bytes = 0;
    for (int q = 0; q < a.nlev; ++q) {
        LevelBuf& lb = c->lv[l0 + q];
        a.lv[q] = TailLevel<T>{lb.g, lb.radius, Prec<T>::coef(lb)};
        a.plane_bytes += tail_plane_values(lb.g.n, q, a.nlev) * (long long)sizeof(cplx<T>);
    }
    // the coarsest inverse is copied to LDS when it fits beside the planes
    // (each visit of the coarsest level then reads it without global round trips)
    long long end = a.plane_bytes;
    auto place = [&](long long bytes) -> long long {
        const long long off = (end + 15) / 16 * 16;
        if (off + bytes > kTailMaxLdsBytes) return -1;
        end = off + bytes;
        return off;
    };
    const long long Nc = (long long)(c->lv[c->L - 1].g.n + 1) * (c->lv[c->L - 1].g.n + 1);
    a.inv_off = c->inv ? place(Nc * Nc * (long long)sizeof(cplx<double>)) : -1;
    a.lds_bytes = end;
    LevelBuf& top = c->lv[l0];
    a.u_top = Prec<T>::u(top);
    a.f_top = Prec<T>::f(top);
    a.inv = c->inv;
    a.gamma = cp.gamma;
    a.smoother = cp.smoother == MG_JACOBI ? 0 : 1;
    a.nu1 = cp.nu1;
    a.nu2 = cp.nu2;
    a.omega = cp.omega;
    a.breakdown = Prec<T>::breakdown;
    a.bez = c->transfer == MG_TRANSFER_BEZIER;
    a.top_zero = top_zero;
    launch_tail<T>(lc, a);
}

// r_ready_nblk > 0: level l was entered with u = 0 and the restriction (or,
// on level 0 of an FP32 cycle, the FP64 residual pass before it) also formed
// the first GMRES residual. u_zero: u itself does not hold those zeros.
// first_visit: level l was entered by the restriction that zeroed its u.
// defer (may be null): the update pass of the last post-smoothing step is left
// to the caller's coarse grid correction (*defer describes it; defer->Z.p is
// null where no update is pending and u holds the result). w_ready (level 0
// of FP32 cycles, with r_ready_nblk): that FP64 pass also formed the first
// product A z_0 of the first GMRES step.
template <typename T>
void cycle(mg_ctx* c, const LaunchCtx& lc, int l, const CycleParams& cp, int r_ready_nblk = 0, bool u_zero = false,
           bool first_visit = false, DeferredUpdate<T>* defer = nullptr, bool w_ready = false) {
    if (l == c->tail_level[sizeof(T) == 4]) {
        launch_tail_from<T>(c, lc, l, cp, first_visit);
        return;
    }
    LevelBuf& lb = c->lv[l];
    if (l == c->L - 1) {
        launch_coarse_solve<T>(lc, lb.g, c->dense, c->piv, vec<T>(Prec<T>::f(lb), lb), vec<T>(Prec<T>::u(lb), lb));
        return;
    }
    LevelBuf& cb = c->lv[l + 1];
    // the next level's first GMRES step starts from its zeroed iterate: its
    // residual pass is the restriction itself (launched levels only)
    const int lc1 = l + 1;
    const bool r_in_restrict = cp.smoother == MG_GMRES3 && cp.nu1 > 0 && lc1 != c->tail_level[sizeof(T) == 4] &&
                               lc1 != c->L - 1;
    RestrictOut<T> ro;
    ro.gc = cb.g;
    ro.transfer = c->transfer;
    ro.fc = vec<T>(Prec<T>::f(cb), cb);
    ro.uc = vec<T>(Prec<T>::u(cb), cb);
    ro.zc = r_in_restrict ? vec<T>(Prec<T>::V(cb), cb) : Vec<T>{nullptr, 0};
    // the last GMRES pre-smoothing step also forms the residual to restrict,
    // and restricts it itself where the handle fuses the two
    const bool fused = cp.smoother == MG_GMRES3 && cp.nu1 > 0;
    // Jacobi sweeps go in pairs (one pass each where the level allows it)
    auto jsteps = [&](int s, int nu) { return cp.smoother == MG_JACOBI && s + 1 < nu ? 2 : 1; };
    for (int s = 0; s < cp.nu1; s += jsteps(s, cp.nu1))
        smooth<T>(c, lc, l, cp, fused && s == cp.nu1 - 1, s == 0 ? r_ready_nblk : 0, ProlongIn<T>{},
                  s == 0 && u_zero, fused && s == cp.nu1 - 1 ? &ro : nullptr, jsteps(s, cp.nu1), nullptr,
                  s == 0 && w_ready);
    if (!fused)
        launch_residual<T>(lc, level_op<T>(c, l), vec<T>(Prec<T>::u(lb), lb), vec<T>(Prec<T>::f(lb), lb),
                           vec<T>(Prec<T>::w(lb), lb));
    const int nb_r = ro.nblk > 0 ? ro.nblk
                                 : launch_restrict<T>(lc, lb.g, cb.g, c->transfer, vec<T>(Prec<T>::w(lb), lb),
                                                      ro.fc, ro.uc, ro.zc);
    // the coarse grid correction u += P e is formed by the first pass of the
    // first post-smoothing GMRES step, into the fourth Arnoldi plane (unused
    // by the step's own passes); on handles for one right-hand side that pass
    // also forms e itself from the pending update of the coarse level's last
    // visit (earlier visits of a W-cycle write their iterate, from which the
    // next visit starts), except on a level-1 product operator. Measured per
    // level at n = 1024: the update pass it replaces costs 5-9 us, the
    // correction pass grows by 3-6 us (the weights' reduction and
    // least-squares solve move onto its critical path), by 13 us on the
    // product operator; batch launches were slower with it.
    const bool pro_fused = cp.smoother == MG_GMRES3 && cp.nu2 > 0;
    const bool defer_coarse =
        pro_fused && c->defer_update && lc.nrhs_cap == 1 && !(l == 1 && level_op<T>(c, 1).product);
    DeferredUpdate<T> du{};
    for (int g = 0; g < cp.gamma; ++g)
        cycle<T>(c, lc, l + 1, cp, g == 0 && r_in_restrict ? nb_r : 0, false, g == 0,
                 defer_coarse && g + 1 == cp.gamma ? &du : nullptr);
    const Vec<T> e = vec<T>(Prec<T>::u(cb), cb);
    if (!pro_fused) launch_prolong_add<T>(lc, cb.g, lb.g, c->transfer, e, vec<T>(Prec<T>::u(lb), lb));
    for (int s = 0; s < cp.nu2; s += jsteps(s, cp.nu2)) {
        ProlongIn<T> pro{};
        if (pro_fused && s == 0) {
            const Vec<T> Z = vec<T>(Prec<T>::V(lb), lb);
            pro = ProlongIn<T>{cb.g, e, c->transfer, Vec<T>{Z.p + 3 * Z.plane, 4 * Z.plane}, du};
        }
        const bool last = s + jsteps(s, cp.nu2) >= cp.nu2;
        smooth<T>(c, lc, l, cp, false, 0, pro, false, nullptr, jsteps(s, cp.nu2), last ? defer : nullptr);
    }
}

// Zeroes every vector and coefficient plane (ghost frames must read zero).
mg_status zero_workspace(mg_ctx* c, hipStream_t s) {
    launch_fill_words(s, c->ws, (long long)(c->ws_bytes / 4 * 4), 0u);
    return check_launch(c);
}

// The k^2 field must be finite, non-negative, and positive on the boundary
// (§2: the absorbing condition takes k = sqrt(k^2) there). Checked on the
// device before the hierarchy is touched; MG_E_ARG with the first offending
// node in *why otherwise.
mg_status check_k2(mg_ctx* c, const double* k2, hipStream_t s, std::string* why) {
    launch_fill_words(s, c->k2_flags, 4, 0u);
    launch_fill_words(s, c->k2_flags + 1, 4, 0x7fffffffu);
    launch_check_k2(s, c->n, k2, c->k2_flags);
    if (mg_status st = check_launch(c)) {
        *why = c->err;
        return st;
    }
    int flags[2] = {0, 0};
    if (hipMemcpyAsync(flags, c->k2_flags, sizeof(flags), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        *why = "k2 check: copy of its result failed";
        return MG_E_HIP;
    }
    if (flags[0] == 0) return MG_OK;
    const int m = c->n + 1;
    const int i = flags[1] % m, j = flags[1] / m;
    std::string what;
    if (flags[0] & 1) what += " non-finite values;";
    if (flags[0] & 2) what += " negative values;";
    if (flags[0] & 4) what += " zeros on the boundary;";
    *why = "k2 must be finite, >= 0 and > 0 on the boundary: found" + what + " first at node (i, j) = (" +
           std::to_string(i) + ", " + std::to_string(j) + ")";
    return MG_E_ARG;
}

// input_read (may be null) is recorded once the caller's k2 has been copied.
mg_status build_hierarchy(mg_ctx* c, const double* k2, hipStream_t s, hipEvent_t input_read = nullptr) {
    const Grid g0 = c->lv[0].g;
    launch_k2_in(s, g0, k2, c->k2_64, c->k2_32);
    if (input_read) HM_HIP(hipEventRecord(input_read, s));
    for (int l = 0; l + 1 < c->L; ++l) {
        const LevelBuf& f = c->lv[l];
        LevelBuf& cc = c->lv[l + 1];
        launch_galerkin(s, l, f.g, f.radius, f.coef64, c->k2_64, c->h, c->shift, c->transfer, cc.g, cc.radius,
                        cc.coef64);
        if (c->has32) {
            const long long nc = (long long)(2 * cc.radius + 1) * (2 * cc.radius + 1) * cc.g.plane;
            launch_cast_coef(s, cc.coef64, cc.coef32, nc);
        }
    }
    const LevelBuf& lc = c->lv[c->L - 1];
    launch_dense_lu(s, lc.g, lc.radius, lc.coef64, c->dense, c->piv);
    if (c->inv) launch_lu_inverse(s, (lc.g.n + 1) * (lc.g.n + 1), c->dense, c->piv, c->inv);
    return check_launch(c);
}

// Levels of at most tail_n intervals (HELMG_TAIL_N, default 16) run in the
// single-workgroup tail when all of them fit its LDS budget at the cycle's
// precision and the coarsest grid is small enough for the explicit inverse;
// HELMG_TAIL_N = 0 turns the tail off.
void pick_tail_levels(mg_ctx* c, int tail_n) {
    const int L = c->L;
    const int nc = c->n >> (L - 1);
    const bool small_coarse = (nc + 1) * (nc + 1) <= kTailMaxCoarseNodes;
    for (int prec = 0; prec < 2; ++prec) {
        const long long elem = prec ? 8 : 16;
        c->tail_level[prec] = -1;
        if (tail_n <= 0 || !small_coarse) continue;
        for (int l = 1; l < L; ++l) {
            if ((c->n >> l) > tail_n || L - l > kMaxTailLevels) continue;
            long long bytes = 0;
            for (int q = 0; q < L - l; ++q) bytes += tail_plane_values(c->n >> (l + q), q, L - l) * elem;
            if (bytes <= kTailMaxLdsBytes) {
                c->tail_level[prec] = l;
                break;
            }
        }
    }
}

bool is_dev_ptr_ok(const void* p) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) % 8) == 0; }

mg_solve_opts default_solve_opts() {
    mg_solve_opts o;
    o.nu_pre = 1;
    o.nu_post = 1;
    o.omega = 4.5;
    o.max_cycles = 500;
    o.precision = MG_FP64;
    o.divergence = 1e8;
    return o;
}

// A caller's history buffer must hold max_cycles entries per right-hand side.
mg_status check_stats(mg_ctx* c, const mg_solve_stats* stats, int nrhs, int max_cycles) {
    if (stats && stats->history && (long long)stats->history_len < (long long)max_cycles * nrhs) {
        c->err = "stats->history_len (" + std::to_string(stats->history_len) + ") < max_cycles * nrhs (" +
                 std::to_string((long long)max_cycles * nrhs) + ")";
        return MG_E_ARG;
    }
    return MG_OK;
}

mg_status check_solve_args(mg_ctx* c, int nrhs, double tol, int cyc, int smoother, const mg_solve_opts& o) {
    if (nrhs < 1 || nrhs > c->max_batch) { c->err = "nrhs must be in [1, max_batch]"; return MG_E_ARG; }
    if (!(tol > 0.0)) { c->err = "tol must be > 0"; return MG_E_ARG; }
    if (cyc != MG_V && cyc != MG_W) { c->err = "cycle must be MG_V or MG_W"; return MG_E_ARG; }
    if (smoother != MG_JACOBI && smoother != MG_GMRES3) { c->err = "unknown smoother"; return MG_E_ARG; }
    if (o.nu_pre < 0 || o.nu_post < 0 || o.nu_pre + o.nu_post > 64) { c->err = "nu out of range"; return MG_E_ARG; }
    if (!(o.omega > 0.0)) { c->err = "omega must be > 0"; return MG_E_ARG; }
    if (o.max_cycles < 1) { c->err = "max_cycles must be >= 1"; return MG_E_ARG; }
    if (o.precision != MG_FP64 && o.precision != MG_FP32_REFINED) { c->err = "unknown precision"; return MG_E_ARG; }
    if (o.precision == MG_FP32_REFINED && !c->has32) {
        c->err = "handle was set up without FP32 copies";
        return MG_E_STATE;
    }
    if (!(o.divergence > 1.0)) { c->err = "divergence factor must be > 1"; return MG_E_ARG; }
    return MG_OK;
}

// Core solve of A_s x = f_s on level-0 buffers: f_s already in lv[0].f64, the
// initial guess in lv[0].u64. Leaves every solution in lv[0].u64.
// One solve on one handle, driven cycle by cycle (§5 stop test): start()
// enqueues the initial norms; after the stream has synchronised, begin()
// reads them and hands the device its stop limits. enqueue_cycle() enqueues
// one cycle and its residual norms with the device-side stop test on a stream
// (captured or eager); enqueued(it) records the buffer state after cycle it,
// and after_cycle(it) reads that cycle's stop-test reports once it has
// completed, so cycles may be queued ahead of the reports. gather() collects
// every right-hand side's last iterate.
struct SolveRun {
    mg_ctx* c = nullptr;
    int nrhs = 0;
    double tol = 0.0;
    CycleParams cp{};
    mg_solve_opts o{};
    bool fp32 = false;
    std::vector<double> rel0, rel, rel_prev;
    std::vector<int> cycles, state;  // state: 0 running, 1 converged, 2 diverged
    std::vector<int> buf_after;      // cur_buf after each enqueued cycle
    int running = 0;
    // FP32 cycles whose first level-0 GMRES residual comes from the FP64
    // residual pass before them (u = 0 is not stored; no zeroing pass), and
    // that pass's partial sums per right-hand side; w_ready: that pass also
    // forms the step's first product A z_0 (one pass fewer per cycle)
    bool z_ready = false;
    bool w_ready = false;
    int z_nblk = 0;
    std::vector<uintptr_t> key;
    std::chrono::steady_clock::time_point t0;

    SolveRun(mg_ctx* ctx, int nr, double tl, int cyc, int smoother, const mg_solve_opts& opts)
        : c(ctx), nrhs(nr), tol(tl), cp{cyc, smoother, opts.nu_pre, opts.nu_post, opts.omega}, o(opts),
          fp32(opts.precision == MG_FP32_REFINED) {
        uint64_t omega_bits;
        std::memcpy(&omega_bits, &o.omega, sizeof(omega_bits));
        key = {uintptr_t(fp32), uintptr_t(cyc), uintptr_t(smoother), uintptr_t(o.nu_pre), uintptr_t(o.nu_post),
               uintptr_t(omega_bits), uintptr_t(nrhs), uintptr_t(c->timing_class)};
    }
    LaunchCtx ctx(hipStream_t s) const { return launch_ctx(c, s, nrhs); }
    Vec<float> z_plane() const {
        LevelBuf& l0 = c->lv[0];
        return z_ready ? vec<float>(Prec<float>::V(l0), l0) : Vec<float>{nullptr, 0};
    }
    Vec<float> w_plane() const {
        LevelBuf& l0 = c->lv[0];
        return w_ready ? vec<float>(Prec<float>::w(l0), l0) : Vec<float>{nullptr, 0};
    }

    mg_status start(hipStream_t s) {
        t0 = std::chrono::steady_clock::now();
        LevelBuf& l0 = c->lv[0];
        const LevelOp<double> op0 = level_op<double>(c, 0);
        c->cur_buf = 0;
        c->final_buf.assign(nrhs, -1);
        for (int b = 0; b < nrhs; ++b) c->h_active[b] = 1;
        HM_HIP(hipMemcpyAsync(c->active, c->h_active, sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
        LaunchCtx lc = ctx(s);
        launch_norm<double>(lc, l0.g, vec<double>(l0.f64, l0), c->norms);
        if (fp32) {
            z_ready = cp.smoother == MG_GMRES3 && cp.nu1 > 0 && c->L > 1 && c->tail_level[1] != 0;
            w_ready = z_ready && c->fuse_r_a0 && refine_apply_fits(lc, l0.g);
            key.push_back(uintptr_t(w_ready));
            z_nblk = launch_refine_residual(lc, op0, vec<double>(l0.u64, l0), vec<double>(l0.f64, l0),
                                            vec<float>(l0.f32, l0), c->norms, z_plane(), c->k2_32, w_plane());
        }
        else
            launch_resnorm<double>(lc, op0, vec<double>(l0.u64, l0), vec<double>(l0.f64, l0), c->norms);
        if (mg_status st = check_launch(c)) return st;
        HM_HIP(hipMemcpyAsync(c->h_norms, c->norms, sizeof(RhsNorms) * nrhs, hipMemcpyDeviceToHost, s));
        return MG_OK;
    }

    mg_status begin(hipStream_t s) {
        LevelBuf& l0 = c->lv[0];
        rel0.assign(nrhs, 0.0);
        rel.assign(nrhs, 0.0);
        rel_prev.assign(nrhs, 0.0);
        cycles.assign(nrhs, 0);
        state.assign(nrhs, 0);
        running = 0;
        for (int b = 0; b < nrhs; ++b) {
            const double f2 = c->h_norms[b].f2;
            if (f2 == 0.0) {
                // zero right-hand side: the solution is zero
                launch_zero<double>(s, l0.u64 + (long long)b * l0.g.plane, l0.g.plane);
                rel0[b] = rel[b] = 0.0;
                state[b] = 1;
            } else {
                rel0[b] = rel[b] = std::sqrt(c->h_norms[b].r2 / f2);
                if (!std::isfinite(rel0[b])) state[b] = 2;
                else if (rel0[b] <= tol) state[b] = 1;
            }
            if (state[b] != 0) {
                c->h_active[b] = 0;
                c->final_buf[b] = 0;
            } else {
                ++running;
            }
        }
        for (int b = 0; b < nrhs; ++b) {
            c->h_limits[2 * b] = tol;
            c->h_limits[2 * b + 1] = o.divergence * rel0[b];
        }
        HM_HIP(hipMemcpyAsync(c->active, c->h_active, sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
        HM_HIP(hipMemcpyAsync(c->stop_limits, c->h_limits, sizeof(double) * 2 * nrhs, hipMemcpyHostToDevice, s));
        HM_HIP(hipMemsetAsync(c->stop_count, 0, sizeof(int) * nrhs, s));
        buf_after.clear();
        return MG_OK;
    }

    void enqueue_cycle(hipStream_t st) {
        LevelBuf& l0 = c->lv[0];
        const LevelOp<double> op0 = level_op<double>(c, 0);
        LaunchCtx l2 = ctx(st);
        // the closing norm pass takes the stop test
        LaunchCtx lt = l2;
        lt.stop = StopTest{c->h_ring, c->active, c->stop_count, c->stop_limits, c->max_batch};
        if (fp32) {
            if (!z_ready) launch_zero<float>(st, l0.u32, l0.g.plane * nrhs);
            cycle<float>(c, l2, 0, cp, z_ready ? z_nblk : 0, z_ready, false, nullptr, w_ready);
            cplx<double>* xin = c->cur_buf == 0 ? l0.u64 : l0.t64;
            cplx<double>* xout = c->cur_buf == 0 ? l0.t64 : l0.u64;
            z_nblk = launch_correct_residual(lt, op0, vec<double>(xin, l0), vec<float>(l0.u32, l0),
                                             vec<double>(xout, l0), vec<double>(l0.f64, l0), vec<float>(l0.f32, l0),
                                             c->norms, z_plane(), c->k2_32, w_plane());
            c->cur_buf ^= 1;
        } else {
            cycle<double>(c, l2, 0, cp);
            launch_resnorm<double>(lt, op0, vec<double>(l0.u64, l0), vec<double>(l0.f64, l0), c->norms);
        }
    }

    // cycle `it` (1-based) has been enqueued (eagerly or as a graph replay),
    // leaving the FP64 iterate in buffer cur
    void enqueued(int it, int cur) {
        if ((int)buf_after.size() < it) buf_after.resize(it, 0);
        buf_after[it - 1] = cur;
    }

    // after cycle `it` has completed: the device's stop decisions and norms.
    // A right-hand side's iterate stays where its stopping cycle left it,
    // since later cycles skip it.
    mg_status after_cycle(int it, mg_solve_stats* stats) {
        harvest_timing(c);
        for (int b = 0; b < nrhs; ++b) {
            if (state[b] != 0) {
                if (stats && stats->history) stats->history[(size_t)(it - 1) * nrhs + b] = NAN;
                continue;
            }
            const RhsReport rep = c->h_ring[((it - 1) % kReportRing) * c->max_batch + b];
            if (rep.cycle != it) {
                c->err = "stop-test report out of sequence";
                return MG_E_HIP;
            }
            const double r = std::sqrt(rep.r2 / rep.f2);
            rel_prev[b] = rel[b];
            rel[b] = r;
            cycles[b] = it;
            if (stats && stats->history) stats->history[(size_t)(it - 1) * nrhs + b] = r;
            if (c->log)
                std::fprintf(stderr, "helmg: handle %p rhs %d cycle %d relres %.6e contraction %.4f%s\n",
                             static_cast<void*>(c), b, it, r, rel_prev[b] > 0.0 ? r / rel_prev[b] : 0.0,
                             rep.stop == 1 ? " converged" : rep.stop == 2 ? " diverged" : "");
            if (rep.stop) {
                state[b] = rep.stop;
                c->h_active[b] = 0;
                c->final_buf[b] = buf_after[it - 1];
                --running;
            }
        }
        return MG_OK;
    }

    // The cycle after which every running right-hand side is expected within
    // twice the tolerance, its relative residual after cycle `it` extrapolated
    // by its last contraction factor (INT_MAX when one does not contract).
    // Cycles queued beyond the last one do no work but still cost most of a
    // cycle's launches, so the host queues ahead only up to this cycle.
    int predicted_last(int it) const {
        int last = it;
        for (int b = 0; b < nrhs; ++b) {
            if (state[b] != 0) continue;
            const double q = rel_prev[b] > 0.0 ? rel[b] / rel_prev[b] : 1.0;
            if (!(q < 1.0)) return INT_MAX;
            int m = 1;
            for (double r = rel[b] * q; r > 2.0 * tol && m < 4096; r *= q) ++m;
            last = std::max(last, it + m);
        }
        return last;
    }

    // enqueues the gather of the final iterates (no synchronisation)
    mg_status gather(hipStream_t s) {
        LevelBuf& l0 = c->lv[0];
        for (int b = 0; b < nrhs; ++b)
            if (c->final_buf[b] < 0) c->final_buf[b] = c->cur_buf;
        if (fp32) {
            // buffer 0 = u64, buffer 1 = t64 (pointers never swapped in this path)
            for (int b = 0; b < nrhs; ++b)
                if (c->final_buf[b] == 1)
                    HM_HIP(hipMemcpyAsync(l0.u64 + (long long)b * l0.g.plane, l0.t64 + (long long)b * l0.g.plane,
                                          size_t(l0.g.plane) * 16, hipMemcpyDeviceToDevice, s));
        } else {
            // Jacobi on level 0 swaps the u64 / t64 pointers (cur_buf counts the
            // parity); a right-hand side that stopped at another parity than the
            // current one has its iterate in t64 now.
            for (int b = 0; b < nrhs; ++b)
                if (c->final_buf[b] != c->cur_buf)
                    HM_HIP(hipMemcpyAsync(l0.u64 + (long long)b * l0.g.plane, l0.t64 + (long long)b * l0.g.plane,
                                          size_t(l0.g.plane) * 16, hipMemcpyDeviceToDevice, s));
        }
        return MG_OK;
    }

    // after gather() and a synchronisation
    mg_status result(mg_solve_stats* stats) {
        mg_status res = MG_OK;
        for (int b = 0; b < nrhs; ++b) {
            if (state[b] == 2) res = MG_E_DIVERGED;
            else if (state[b] == 0 && res == MG_OK) res = MG_NOT_CONVERGED;
        }
        if (stats) {
            for (int b = 0; b < nrhs; ++b) {
                if (stats->cycles) stats->cycles[b] = cycles[b];
                if (stats->relres) stats->relres[b] = rel[b];
            }
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        if (res == MG_E_DIVERGED) c->err = "residual diverged";
        return res;
    }
};

mg_status solve_core(mg_ctx* c, hipStream_t s, int nrhs, double tol, int cyc, int smoother, const mg_solve_opts& o,
                     mg_solve_stats* stats) {
    SolveRun run(c, nrhs, tol, cyc, smoother, o);
    if (mg_status st = run.start(s)) return st;
    HM_HIP(hipStreamSynchronize(s));
    if (mg_status st = run.begin(s)) return st;
    // Cycles are launched in groups of one or two (one captured graph and one
    // completion event per group: each graph launch costs a gap of about 13 us
    // on the GPU), and a second group is queued behind the one whose reports
    // the host waits for, so the GPU does not idle through the host's
    // turn-around. Both only up to the cycle at which the solve is expected to
    // end (predicted_last); the next cycle is always queued. Per-kernel timing
    // (eager launches with events) runs one cycle at a time.
    const bool may_run_ahead = c->timing_class == 0;
    struct Group {
        int last;  // its cycles end with this one
        int ev;
    };
    Group inflight[2];
    int n_inflight = 0, ev_next = 0, it = 0, enq = 0;
    auto launch = [&](int count) -> mg_status {
        std::vector<uintptr_t> key = run.key;
        key.push_back(uintptr_t(count));
        auto body = [&](hipStream_t st) {
            for (int q = 0; q < count; ++q) {
                run.enqueue_cycle(st);
                c->graph_marks.push_back(c->cur_buf);
            }
        };
        if (mg_status st = run_cycle_graph(c, s, key, body)) return st;
        if (mg_status st = check_launch(c)) return st;
        for (int q = 0; q < count; ++q) run.enqueued(enq + 1 + q, c->graph_marks[q]);
        enq += count;
        HM_HIP(hipEventRecord(c->cycle_done[ev_next], s));
        inflight[n_inflight++] = Group{enq, ev_next};
        ev_next ^= 1;
        return MG_OK;
    };
    while (run.running > 0 && it < o.max_cycles) {
        const int plast = may_run_ahead ? run.predicted_last(it) : it + 1;
        while (n_inflight < 2 && enq < o.max_cycles && (enq == it || (may_run_ahead && enq < plast))) {
            const int count = (may_run_ahead && enq + 2 <= plast && enq + 2 <= o.max_cycles) ? 2 : 1;
            if (mg_status st = launch(count)) return st;
        }
        const Group g = inflight[0];
        inflight[0] = inflight[1];
        --n_inflight;
        HM_HIP(hipEventSynchronize(c->cycle_done[g.ev]));
        while (it < g.last && run.running > 0) {
            ++it;
            if (mg_status st = run.after_cycle(it, stats)) return st;
        }
    }
    if (mg_status st = run.gather(s)) return st;
    HM_HIP(hipStreamSynchronize(s));
    return run.result(stats);
}

mg_status check_level(mg_ctx* c, int level, int precision, bool allow_last) {
    if (level < 0 || level >= c->L || (!allow_last && level == c->L - 1)) {
        c->err = "level out of range";
        return MG_E_ARG;
    }
    if (precision != MG_FP64 && precision != MG_FP32_REFINED) { c->err = "unknown precision"; return MG_E_ARG; }
    if (precision == MG_FP32_REFINED && !c->has32) { c->err = "no FP32 copies"; return MG_E_STATE; }
    return MG_OK;
}

}  // namespace

// ======================================================================= C ABI
extern "C" {

size_t mg_workspace_bytes(int n, int levels, int transfer, const mg_setup_opts* opts) {
    const int max_batch = opts ? opts->max_batch : 1;
    const int coarsest_n = (opts && opts->coarsest_n > 0) ? opts->coarsest_n : 4;
    const int has32 = opts ? (opts->precision == MG_FP32_REFINED) : 0;
    if (max_batch < 1 || (transfer != MG_TRANSFER_BEZIER && transfer != MG_TRANSFER_LINEAR)) return 0;
    int L;
    std::string why;
    if (!levels_for(n, levels, coarsest_n, &L, &why)) return 0;
    return carve(nullptr, nullptr, n, L, transfer, max_batch, has32);
}

mg_status mg_setup(const double* k2, int n, double h, double shift, int levels, int transfer,
                   const mg_setup_opts* opts, void* workspace, size_t ws_bytes, void* stream, mg_handle* out) {
    if (!out) { g_setup_error = "out is NULL"; return MG_E_ARG; }
    *out = nullptr;
    const int max_batch = opts ? opts->max_batch : 1;
    const int coarsest_n = (opts && opts->coarsest_n > 0) ? opts->coarsest_n : 4;
    const int has32 = opts ? (opts->precision == MG_FP32_REFINED) : 0;
    if (!is_dev_ptr_ok(k2)) { g_setup_error = "k2 is NULL or misaligned"; return MG_E_ARG; }
    if (!(h > 0.0) || !std::isfinite(h)) { g_setup_error = "h must be > 0"; return MG_E_ARG; }
    if (!(shift >= 0.0) || !std::isfinite(shift)) { g_setup_error = "shift must be >= 0"; return MG_E_ARG; }
    if (transfer != MG_TRANSFER_BEZIER && transfer != MG_TRANSFER_LINEAR) { g_setup_error = "bad transfer"; return MG_E_ARG; }
    if (max_batch < 1 || max_batch > 4096) { g_setup_error = "max_batch out of range"; return MG_E_ARG; }
    if (opts && opts->precision != MG_FP64 && opts->precision != MG_FP32_REFINED) {
        g_setup_error = "unknown precision";
        return MG_E_ARG;
    }
    int L;
    if (!levels_for(n, levels, coarsest_n, &L, &g_setup_error)) return MG_E_ARG;
    const size_t need = carve(nullptr, nullptr, n, L, transfer, max_batch, has32);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) {
        g_setup_error = "workspace is NULL or not 256-byte aligned";
        return MG_E_WORKSPACE;
    }
    if (ws_bytes < need) {
        g_setup_error = "workspace too small: need " + std::to_string(need) + " bytes";
        return MG_E_WORKSPACE;
    }
    mg_ctx* c = new mg_ctx();
    c->n = n;
    c->L = L;
    c->transfer = transfer;
    c->max_batch = max_batch;
    c->has32 = has32;
    c->coarsest_n = coarsest_n;
    c->h = h;
    c->shift = shift;
    c->ws = static_cast<char*>(workspace);
    c->ws_bytes = need;
    if (const char* e = std::getenv("HELMG_GRAPH")) c->use_graph = std::atoi(e) != 0;
    if (opts && opts->use_graph < 0) c->use_graph = false;
    if (opts && opts->tune_cache) c->tune_cache = opts->tune_cache;
    if (const char* e = std::getenv("HELMG_TALL_BLOCKS")) {
        const int v = std::atoi(e);
        c->tall_rows = (v == 8 || v == 16) ? v : 4;
    }
    if (const char* e = std::getenv("HELMG_SMALL_ROWS")) c->small_rows = std::atoi(e) == 4 ? 4 : 2;
    if (const char* e = std::getenv("HELMG_L1_PRODUCT")) c->product_l1 = std::atoi(e);
    if (const char* e = std::getenv("HELMG_FUSE_CORRECTION")) c->fuse_correction = std::atoi(e) != 0;
    if (const char* e = std::getenv("HELMG_FUSE_RESTRICT")) c->fuse_restrict = std::atoi(e) != 0;
    if (const char* e = std::getenv("HELMG_FUSE_R_A0")) c->fuse_r_a0 = std::atoi(e) != 0;
    if (const char* e = std::getenv("HELMG_LOG")) c->log = std::atoi(e) != 0;
    if (const char* e = std::getenv("HELMG_JACOBI_PAIRS")) c->jacobi_pairs = std::atoi(e) != 0;
    if (const char* e = std::getenv("HELMG_DEFER_UPDATE")) c->defer_update = std::atoi(e) != 0;
    // batch handles: fewer, larger tiles per right-hand side (the launch has
    // max_batch times as many blocks; larger tiles amortise each block's
    // fixed costs: reduction, tile halo, block sums)
    if (max_batch > 1) c->block_cap = std::max(64, 640 / max_batch);
    if (const char* e = std::getenv("HELMG_MAX_BLOCKS")) {
        const int v = std::atoi(e);
        // room below kMaxPartialBlocks for the rounding of the grid to whole
        // tiles and for the padding of batch grids to multiples of 8 tiles
        constexpr int kCapMax = kMaxPartialBlocks - 1024;
        c->block_cap = v < 64 ? 64 : (v > kCapMax ? kCapMax : v);
    }
    {
        // default tail: levels of at most 16 intervals (the autotuner's choice on
        // the n = 1024 benchmark; 32 was 0.5 ms per solve slower there)
        int tail_n = 16;
        if (const char* e = std::getenv("HELMG_TAIL_N")) tail_n = std::atoi(e);
        c->tail_n = tail_n;
        pick_tail_levels(c, tail_n);
    }
    tail_init();
    {
        // the device and, once per device, the address of the static scratch
        // of mg_residual_noalloc (looked up here, at set-up, with the device current)
        void* scr = nullptr;
        hipError_t e = hipGetDevice(&c->device);
        if (e == hipSuccess) e = static_scratch(c->device, &scr);
        if (e != hipSuccess) {
            g_setup_error = std::string("device scratch lookup: ") + hipGetErrorString(e);
            delete c;
            return MG_E_HIP;
        }
    }
    carve(c, c->ws, n, L, transfer, max_batch, has32);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_norms), sizeof(RhsNorms) * max_batch, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_active), sizeof(int) * max_batch, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_limits), sizeof(double) * 2 * max_batch, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->h_ring), sizeof(RhsReport) * kReportRing * max_batch,
                      hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->cycle_done[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->cycle_done[1], hipEventDisableTiming) != hipSuccess) {
        g_setup_error = "pinned host buffers or events could not be created";
        mg_destroy(c);
        return MG_E_HIP;
    }
    mg_status st = zero_workspace(c, s);
    if (st == MG_OK) {
        std::string why;
        st = check_k2(c, k2, s, &why);
        if (st != MG_OK) {
            g_setup_error = why;
            mg_destroy(c);
            return st;
        }
    }
    if (st == MG_OK) st = build_hierarchy(c, k2, s);
    if (st == MG_OK && hipStreamSynchronize(s) != hipSuccess) {
        c->err = "setup synchronisation failed";
        st = MG_E_HIP;
    }
    if (st != MG_OK) {
        g_setup_error = c->err;
        mg_destroy(c);
        return st;
    }
    *out = c;
    return MG_OK;
}

mg_status mg_update_k2(mg_handle c, const double* k2, void* stream) {
    if (!c) return MG_E_ARG;
    if (!is_dev_ptr_ok(k2)) { c->err = "k2 is NULL or misaligned"; return MG_E_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    {
        std::string why;
        if (mg_status st = check_k2(c, k2, s, &why)) {
            c->err = why;
            return st;
        }
    }
    // returns once the caller's k2 has been copied; the Galerkin products and
    // the coarsest factorisation stay queued on the stream ahead of the
    // caller's next work (an event slot of the solve loop, idle between calls)
    if (mg_status st = build_hierarchy(c, k2, s, c->cycle_done[0])) return st;
    HM_HIP(hipEventSynchronize(c->cycle_done[0]));
    return MG_OK;
}

mg_status mg_solve(mg_handle c, const void* rhs, void* x, int nrhs, double tol, int cyc, int smoother,
                   const mg_solve_opts* opts, mg_solve_stats* stats, void* stream) {
    if (!c) return MG_E_ARG;
    const mg_solve_opts o = opts ? *opts : default_solve_opts();
    if (mg_status st = check_solve_args(c, nrhs, tol, cyc, smoother, o)) return st;
    if (mg_status st = check_stats(c, stats, nrhs, o.max_cycles)) return st;
    if (!is_dev_ptr_ok(rhs) || !is_dev_ptr_ok(x)) { c->err = "rhs / x NULL or misaligned"; return MG_E_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    LevelBuf& l0 = c->lv[0];
    LaunchCtx lc = launch_ctx(c, s, nrhs);
    lc.active = nullptr;
    launch_copy_in<double>(lc, l0.g, rhs, false, vec<double>(l0.f64, l0), true, false);
    launch_copy_in<double>(lc, l0.g, x, false, vec<double>(l0.u64, l0), false, false);
    if (mg_status st = check_launch(c)) return st;
    const mg_status res = solve_core(c, s, nrhs, tol, cyc, smoother, o, stats);
    if (res == MG_E_HIP || res == MG_E_ARG) return res;
    launch_copy_out<double>(lc, l0.g, vec<double>(l0.u64, l0), x, false, false, false);
    if (mg_status st = check_launch(c)) return st;
    HM_HIP(hipStreamSynchronize(s));
    return res;
}

namespace {

// Graphs of mg_solve_multi: one per set of running problems and their buffer
// assignment, alive for one call.
struct MultiGraphs {
    struct Entry {
        std::vector<uintptr_t> key;
        hipGraphExec_t exec = nullptr;
        std::vector<std::vector<void*>> after_ptrs;
        std::vector<int> after_cur;
    };
    std::vector<Entry> entries;
    std::vector<hipStream_t> branch;
    std::vector<hipEvent_t> join;
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr;
    ~MultiGraphs() {
        for (Entry& e : entries)
            if (e.exec) (void)hipGraphExecDestroy(e.exec);
        for (hipStream_t b : branch) (void)hipStreamDestroy(b);
        for (hipEvent_t e : join) (void)hipEventDestroy(e);
        if (cap) (void)hipStreamDestroy(cap);
        if (fork) (void)hipEventDestroy(fork);
    }
    bool ready(size_t nbranch) {
        if (!cap && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return false;
        if (!fork && hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return false;
        while (branch.size() < nbranch) {
            hipStream_t b;
            hipEvent_t e;
            if (hipStreamCreateWithFlags(&b, hipStreamNonBlocking) != hipSuccess) return false;
            branch.push_back(b);
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return false;
            join.push_back(e);
        }
        return true;
    }
};

}  // namespace

mg_status mg_solve_multi(mg_handle* handles, int nprob, const void* const* rhs, void* const* x, const int* nrhs,
                         double tol, int cyc, int smoother, const mg_solve_opts* opts, mg_solve_stats* stats,
                         void* stream) {
    if (!handles || nprob < 1 || !rhs || !x || !nrhs) {
        g_setup_error = "handles, rhs, x and nrhs must be non-NULL and nprob >= 1";
        return MG_E_ARG;
    }
    const mg_solve_opts o = opts ? *opts : default_solve_opts();
    for (int p = 0; p < nprob; ++p) {
        mg_ctx* c = handles[p];
        if (!c) { g_setup_error = "NULL handle"; return MG_E_ARG; }
        for (int q = 0; q < p; ++q)
            if (handles[q] == c) { g_setup_error = "handles must be distinct"; return MG_E_ARG; }
        if (mg_status st = check_solve_args(c, nrhs[p], tol, cyc, smoother, o)) return st;
        if (mg_status st = check_stats(c, stats ? stats + p : nullptr, nrhs[p], o.max_cycles)) return st;
        if (!is_dev_ptr_ok(rhs[p]) || !is_dev_ptr_ok(x[p])) { c->err = "rhs / x NULL or misaligned"; return MG_E_ARG; }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    mg_ctx* c = handles[0];  // carries the message of a stream-level HIP error
    std::vector<SolveRun> runs;
    runs.reserve(nprob);
    for (int p = 0; p < nprob; ++p) {
        mg_ctx* cp = handles[p];
        LevelBuf& l0 = cp->lv[0];
        LaunchCtx lc = launch_ctx(cp, s, nrhs[p]);
        lc.active = nullptr;
        launch_copy_in<double>(lc, l0.g, rhs[p], false, vec<double>(l0.f64, l0), true, false);
        launch_copy_in<double>(lc, l0.g, x[p], false, vec<double>(l0.u64, l0), false, false);
        if (mg_status st = check_launch(cp)) return st;
        runs.emplace_back(cp, nrhs[p], tol, cyc, smoother, o);
        if (mg_status st = runs.back().start(s)) return st;
    }
    HM_HIP(hipStreamSynchronize(s));
    for (SolveRun& r : runs)
        if (mg_status st = r.begin(s)) return st;
    bool use_graph = true;
    for (SolveRun& r : runs) use_graph = use_graph && r.c->use_graph && r.c->timing_class == 0;
    MultiGraphs mg;
    int it = 0;
    for (;;) {
        std::vector<int> R;
        for (int p = 0; p < nprob; ++p)
            if (runs[p].running > 0) R.push_back(p);
        if (R.empty() || it >= o.max_cycles) break;
        ++it;
        bool launched = false;
        if (use_graph) {
            std::vector<uintptr_t> key;
            for (int p : R) {
                mg_ctx* cp = runs[p].c;
                key.push_back(uintptr_t(p));
                key.insert(key.end(), runs[p].key.begin(), runs[p].key.end());
                for (void* q : pointer_state(cp)) key.push_back(reinterpret_cast<uintptr_t>(q));
                key.push_back(uintptr_t(cp->cur_buf));
            }
            for (MultiGraphs::Entry& e : mg.entries) {
                if (e.key != key) continue;
                for (size_t k = 0; k < R.size(); ++k) {
                    restore_pointer_state(runs[R[k]].c, e.after_ptrs[k]);
                    runs[R[k]].c->cur_buf = e.after_cur[k];
                }
                HM_HIP(hipGraphLaunch(e.exec, s));
                launched = true;
                break;
            }
            if (!launched) {
                std::vector<std::vector<void*>> before;
                std::vector<int> cur_before;
                for (int p : R) {
                    before.push_back(pointer_state(runs[p].c));
                    cur_before.push_back(runs[p].c->cur_buf);
                }
                hipGraph_t graph = nullptr;
                hipGraphExec_t exec = nullptr;
                bool ok = mg.ready(R.size()) &&
                          hipStreamBeginCapture(mg.cap, hipStreamCaptureModeRelaxed) == hipSuccess;
                if (ok) {
                    ok = hipEventRecord(mg.fork, mg.cap) == hipSuccess;
                    for (size_t k = 0; ok && k < R.size(); ++k) {
                        ok = hipStreamWaitEvent(mg.branch[k], mg.fork, 0) == hipSuccess;
                        if (ok) runs[R[k]].enqueue_cycle(mg.branch[k]);
                        ok = ok && hipEventRecord(mg.join[k], mg.branch[k]) == hipSuccess &&
                             hipStreamWaitEvent(mg.cap, mg.join[k], 0) == hipSuccess;
                    }
                    const bool ended = hipStreamEndCapture(mg.cap, &graph) == hipSuccess && graph != nullptr;
                    ok = ok && ended;
                }
                if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
                if (ok) {
                    MultiGraphs::Entry e;
                    e.key = std::move(key);
                    e.exec = exec;
                    for (int p : R) {
                        e.after_ptrs.push_back(pointer_state(runs[p].c));
                        e.after_cur.push_back(runs[p].c->cur_buf);
                    }
                    mg.entries.push_back(std::move(e));
                    HM_HIP(hipGraphLaunch(mg.entries.back().exec, s));
                    launched = true;
                } else {
                    // capture failed: eager launches from here on
                    use_graph = false;
                    for (size_t k = 0; k < R.size(); ++k) {
                        restore_pointer_state(runs[R[k]].c, before[k]);
                        runs[R[k]].c->cur_buf = cur_before[k];
                    }
                }
            }
        }
        if (!launched)
            for (int p : R) runs[p].enqueue_cycle(s);
        for (int p : R) {
            if (mg_status st = check_launch(runs[p].c)) return st;
            runs[p].enqueued(it, runs[p].c->cur_buf);
        }
        HM_HIP(hipStreamSynchronize(s));
        for (int p : R)
            if (mg_status st = runs[p].after_cycle(it, stats ? stats + p : nullptr)) return st;
    }
    for (SolveRun& r : runs)
        if (mg_status st = r.gather(s)) return st;
    HM_HIP(hipStreamSynchronize(s));
    mg_status worst = MG_OK;
    auto rank = [](mg_status st) { return st == MG_OK ? 0 : st == MG_NOT_CONVERGED ? 1 : st == MG_E_DIVERGED ? 2 : 3; };
    for (int p = 0; p < nprob; ++p) {
        const mg_status st = runs[p].result(stats ? stats + p : nullptr);
        if (rank(st) > rank(worst)) worst = st;
        mg_ctx* cp = handles[p];
        LevelBuf& l0 = cp->lv[0];
        LaunchCtx lc = launch_ctx(cp, s, nrhs[p]);
        lc.active = nullptr;
        launch_copy_out<double>(lc, l0.g, vec<double>(l0.u64, l0), x[p], false, false, false);
        if (mg_status st2 = check_launch(cp)) return st2;
    }
    HM_HIP(hipStreamSynchronize(s));
    return worst;
}

namespace {

// Carve of the caller's FGMRES buffer (base == nullptr only measures).
struct KrylovBuf {
    cplx<double>* V = nullptr;  // (m + 1) vectors
    cplx<double>* Z = nullptr;  // m vectors
    cplx<double>* X = nullptr;
    cplx<double>* F = nullptr;
    cplx<double>* Wv = nullptr;
    cplx<double>* H = nullptr;  // [B][m + 1], one column at a time
    cplx<double>* Y = nullptr;  // [B][m]
    long long vstride = 0;      // values per vector (all right-hand sides)
    size_t bytes = 0;
};

KrylovBuf krylov_carve(const mg_ctx* c, int m, char* base) {
    KrylovBuf k;
    Carver cv{base};
    const size_t B = size_t(c->max_batch);
    const size_t pl = size_t(c->lv[0].g.plane);
    k.vstride = (long long)(B * pl);
    k.V = cv.take<cplx<double>>(size_t(m + 1) * B * pl * 16);
    k.Z = cv.take<cplx<double>>(size_t(m) * B * pl * 16);
    k.X = cv.take<cplx<double>>(B * pl * 16);
    k.F = cv.take<cplx<double>>(B * pl * 16);
    k.Wv = cv.take<cplx<double>>(B * pl * 16);
    k.H = cv.take<cplx<double>>(B * size_t(m + 1) * 16);
    k.Y = cv.take<cplx<double>>(B * size_t(m) * 16);
    k.bytes = align_up(cv.off, kAlign);
    return k;
}

}  // namespace

size_t mg_fgmres_workspace_bytes(mg_handle c, int m) {
    if (!c || m < 1 || m > kMaxRestart) return 0;
    return krylov_carve(c, m, nullptr).bytes;
}

mg_status mg_solve_fgmres(mg_handle c, const void* rhs, void* x, int nrhs, double tol, int m, int cyc, int smoother,
                          const mg_solve_opts* opts, void* krylov, size_t krylov_bytes, mg_solve_stats* stats,
                          void* stream) {
    if (!c) return MG_E_ARG;
    const mg_solve_opts o = opts ? *opts : default_solve_opts();
    if (mg_status st = check_solve_args(c, nrhs, tol, cyc, smoother, o)) return st;
    if (m < 1 || m > kMaxRestart) { c->err = "restart length m must be in [1, 64]"; return MG_E_ARG; }
    if (mg_status st = check_stats(c, stats, nrhs, o.max_cycles)) return st;
    if (!is_dev_ptr_ok(rhs) || !is_dev_ptr_ok(x)) { c->err = "rhs / x NULL or misaligned"; return MG_E_ARG; }
    if (!krylov || (reinterpret_cast<uintptr_t>(krylov) % kAlign) != 0) {
        c->err = "krylov buffer NULL or not 256-byte aligned";
        return MG_E_WORKSPACE;
    }
    const KrylovBuf K = krylov_carve(c, m, static_cast<char*>(krylov));
    if (krylov_bytes < K.bytes) {
        c->err = "krylov buffer too small: need " + std::to_string(K.bytes) + " bytes";
        return MG_E_WORKSPACE;
    }
    if (!c->h_hcol) {
        if (hipHostMalloc(reinterpret_cast<void**>(&c->h_hcol),
                          sizeof(cplx<double>) * 2 * c->max_batch * (kMaxRestart + 1), hipHostMallocDefault) !=
                hipSuccess ||
            hipEventCreateWithFlags(&c->hcol_done[0], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->hcol_done[1], hipEventDisableTiming) != hipSuccess) {
            c->err = "pinned host buffer or event for the Hessenberg columns could not be created";
            return MG_E_HIP;
        }
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = static_cast<hipStream_t>(stream);
    LevelBuf& l0 = c->lv[0];
    const Grid g0 = l0.g;
    const long long pl = g0.plane;
    const bool fp32 = o.precision == MG_FP32_REFINED;
    const LevelOp<double> op0 = level_op<double>(c, 0);
    const CycleParams cp{cyc, smoother, o.nu_pre, o.nu_post, o.omega};
    LaunchCtx lc = launch_ctx(c, s, nrhs);
    lc.active = nullptr;
    // every plane of the buffer gets a zero ghost frame (the level-0 operator
    // reads ghosts as zero; kernels here write interior nodes only)
    launch_fill_words(s, krylov, (long long)(K.bytes / 4 * 4), 0u);
    launch_copy_in<double>(lc, g0, rhs, false, vec<double>(K.F, l0), true, false);
    launch_copy_in<double>(lc, g0, x, false, vec<double>(K.X, l0), false, false);
    for (int b = 0; b < nrhs; ++b) c->h_active[b] = 1;
    HM_HIP(hipMemcpyAsync(c->active, c->h_active, sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
    lc.active = c->active;
    launch_norm<double>(lc, g0, vec<double>(K.F, l0), c->norms);
    if (mg_status st = check_launch(c)) return st;
    HM_HIP(hipMemcpyAsync(c->h_norms, c->norms, sizeof(RhsNorms) * nrhs, hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    std::vector<double> nf(nrhs), rel(nrhs, 0.0);
    std::vector<int> its(nrhs, 0), state(nrhs, 0);  // 0 running, 1 converged, 3 out of iterations
    for (int b = 0; b < nrhs; ++b) nf[b] = std::sqrt(c->h_norms[b].f2);
    uint64_t omega_bits;
    std::memcpy(&omega_bits, &o.omega, sizeof(omega_bits));
    // FP32 preconditioner cycles whose first level-0 GMRES residual is the
    // complex64 basis vector itself (u = 0): the pass that writes v_j also
    // writes it as the first Arnoldi vector with its partial norms (z_nblk
    // blocks), so the cycle has no zeroing pass and no level-0 residual pass
    const bool z_ready = fp32 && cp.smoother == MG_GMRES3 && cp.nu1 > 0 && c->L > 1 && c->tail_level[1] != 0;
    cplx<float>* z32 = z_ready ? Prec<float>::V(l0) : nullptr;
    int z_nblk = 0;
    const std::vector<uintptr_t> key{0xF6E5u, uintptr_t(fp32), uintptr_t(cyc), uintptr_t(smoother),
                                     uintptr_t(o.nu_pre), uintptr_t(o.nu_post), uintptr_t(omega_bits),
                                     uintptr_t(nrhs), uintptr_t(z_ready)};
    auto precond_body = [&](hipStream_t st) {
        LaunchCtx l2 = lc;
        l2.stream = st;
        if (fp32) {
            if (!z_ready) launch_zero<float>(st, l0.u32, pl * nrhs);
            cycle<float>(c, l2, 0, cp, z_ready ? z_nblk : 0, z_ready);
        } else {
            launch_zero<double>(st, l0.u64, pl * nrhs);
            cycle<double>(c, l2, 0, cp);
        }
    };
    std::vector<cplx<double>> yh(size_t(nrhs) * m);
    // per right-hand side: Hessenberg columns rotated to upper triangular, rotations, g
    std::vector<std::vector<std::complex<double>>> R(nrhs), gvec(nrhs), sn(nrhs);
    std::vector<std::vector<double>> cs(nrhs);
    std::vector<int> kdir(nrhs, 0);
    auto set_active = [&](const std::vector<int>& act) -> mg_status {
        // an earlier upload from h_active may still be pending on the stream
        HM_HIP(hipStreamSynchronize(s));
        for (int b = 0; b < nrhs; ++b) c->h_active[b] = act[b];
        HM_HIP(hipMemcpyAsync(c->active, c->h_active, sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
        return MG_OK;
    };
    for (;;) {
        // true residual r = f - A x at the start of a restart cycle
        std::vector<int> act(nrhs);
        for (int b = 0; b < nrhs; ++b) act[b] = state[b] == 0;
        if (mg_status st = set_active(act)) return st;
        launch_residual<double>(lc, op0, vec<double>(K.X, l0), vec<double>(K.F, l0), vec<double>(K.Wv, l0));
        launch_resnorm<double>(lc, op0, vec<double>(K.X, l0), vec<double>(K.F, l0), c->norms);
        if (mg_status st = check_launch(c)) return st;
        HM_HIP(hipMemcpyAsync(c->h_norms, c->norms, sizeof(RhsNorms) * nrhs, hipMemcpyDeviceToHost, s));
        HM_HIP(hipStreamSynchronize(s));
        int running = 0;
        for (int b = 0; b < nrhs; ++b) {
            if (state[b] != 0) continue;
            const double beta = std::sqrt(c->h_norms[b].r2);
            rel[b] = nf[b] > 0.0 ? beta / nf[b] : 0.0;
            if (nf[b] == 0.0 || rel[b] <= tol) state[b] = 1;
            else if (its[b] >= o.max_cycles) state[b] = 3;
            if (state[b] != 0) {
                act[b] = 0;
                continue;
            }
            ++running;
            R[b].assign(size_t(m + 1) * m, 0.0);
            gvec[b].assign(m + 1, 0.0);
            gvec[b][0] = beta;
            cs[b].assign(m, 0.0);
            sn[b].assign(m, 0.0);
            kdir[b] = 0;
        }
        if (running == 0) break;
        if (mg_status st = set_active(act)) return st;
        // v_0, and each v_{j+1} below, is also written in complex64 to the
        // FP32 cycle's right-hand side plane when the preconditioner is the
        // FP32 cycle
        z_nblk = launch_kry_first(lc, g0, K.Wv, K.V, pl, c->norms, fp32 ? l0.f32 : nullptr, z32);
        std::vector<int> in_cycle = act;  // right-hand sides updated at the end of this cycle
        std::vector<int> stopped(nrhs, 0);
        // iteration j on the stream: z_j = M(v_j), one cycle from zero on
        // A_s z = v_j; w = A_s z_j orthogonalised into column j of H and
        // v_{j+1}; the column copied to host slot j % 2
        auto enqueue = [&](int j) -> mg_status {
            cplx<double>* vj = K.V + j * K.vstride;
            cplx<double>* zj = K.Z + j * K.vstride;
            if (!fp32) HM_HIP(hipMemcpyAsync(l0.f64, vj, size_t(pl) * nrhs * 16, hipMemcpyDeviceToDevice, s));
            if (mg_status st = run_cycle_graph(c, s, key, precond_body)) return st;
            if (fp32) {
                launch_apply_widened(lc, op0, vec<float>(l0.u32, l0), vec<double>(zj, l0), vec<double>(K.Wv, l0));
            } else {
                HM_HIP(hipMemcpyAsync(zj, l0.u64, size_t(pl) * nrhs * 16, hipMemcpyDeviceToDevice, s));
                launch_apply<double>(lc, op0, vec<double>(zj, l0), vec<double>(K.Wv, l0));
            }
            launch_kry_orthogonalise(lc, g0, K.V, K.vstride, j, K.Wv, K.H, m + 1, pl, fp32 ? l0.f32 : nullptr,
                                     z32);
            if (mg_status st = check_launch(c)) return st;
            HM_HIP(hipMemcpyAsync(c->h_hcol + size_t(j & 1) * nrhs * (m + 1), K.H,
                                  sizeof(cplx<double>) * nrhs * (m + 1), hipMemcpyDeviceToHost, s));
            HM_HIP(hipEventRecord(c->hcol_done[j & 1], s));
            return MG_OK;
        };
        if (mg_status st = enqueue(0)) return st;
        for (int j = 0; j < m; ++j) {
            // iteration j + 1 needs device data only, so it is queued before
            // column j is read; when column j stops a right-hand side, its
            // share of iteration j + 1 is computed but never used (columns
            // beyond kdir are not read), and when it stops all of them the
            // whole iteration is
            if (j + 1 < m)
                if (mg_status st = enqueue(j + 1)) return st;
            HM_HIP(hipEventSynchronize(c->hcol_done[j & 1]));
            const cplx<double>* hcol = c->h_hcol + size_t(j & 1) * nrhs * (m + 1);
            bool any = false, changed = false;
            for (int b = 0; b < nrhs; ++b) {
                if (!act[b]) continue;
                std::vector<std::complex<double>> h(j + 2);
                for (int i = 0; i <= j + 1; ++i) h[i] = {hcol[size_t(b) * (m + 1) + i].re, hcol[size_t(b) * (m + 1) + i].im};
                // earlier rotations, then the one that zeroes h[j+1]
                for (int i = 0; i < j; ++i) {
                    const std::complex<double> a = h[i], bb = h[i + 1];
                    h[i] = cs[b][i] * a + sn[b][i] * bb;
                    h[i + 1] = -std::conj(sn[b][i]) * a + cs[b][i] * bb;
                }
                const std::complex<double> a = h[j], bb = h[j + 1];
                const double na = std::abs(a), rho = std::sqrt(std::norm(a) + std::norm(bb));
                double cj;
                std::complex<double> sj;
                if (rho == 0.0) {
                    cj = 1.0;
                    sj = 0.0;
                } else if (na == 0.0) {
                    cj = 0.0;
                    sj = std::conj(bb) / rho;
                } else {
                    cj = na / rho;
                    sj = (a / na) * std::conj(bb) / rho;
                }
                cs[b][j] = cj;
                sn[b][j] = sj;
                h[j] = cj * a + sj * bb;
                for (int i = 0; i <= j; ++i) R[b][size_t(i) * m + j] = h[i];
                const std::complex<double> g0v = gvec[b][j];
                gvec[b][j] = cj * g0v;
                gvec[b][j + 1] = -std::conj(sj) * g0v;
                const double est = std::abs(gvec[b][j + 1]) / nf[b];
                ++its[b];
                kdir[b] = j + 1;
                rel[b] = est;
                if (stats && stats->history && its[b] <= o.max_cycles)
                    stats->history[size_t(its[b] - 1) * nrhs + b] = est;
                const bool subzero = hcol[size_t(b) * (m + 1) + j + 1].re == 0.0;
                if (est <= tol || its[b] >= o.max_cycles || subzero) {
                    act[b] = 0;
                    changed = true;
                    if (est <= tol) stopped[b] = 1;
                } else {
                    any = true;
                }
            }
            if (!any || j == m - 1) break;
            // takes effect from iteration j + 2 (j + 1 is already queued)
            if (changed)
                if (mg_status st = set_active(act)) return st;
        }
        // x += Z y for every right-hand side of this cycle (R y = g by back substitution)
        for (int b = 0; b < nrhs; ++b) {
            for (int i = 0; i < m; ++i) yh[size_t(b) * m + i] = {0.0, 0.0};
            if (!in_cycle[b]) continue;
            const int k = kdir[b];
            std::vector<std::complex<double>> y(k);
            for (int i = k - 1; i >= 0; --i) {
                std::complex<double> t = gvec[b][i];
                for (int q = i + 1; q < k; ++q) t -= R[b][size_t(i) * m + q] * y[q];
                y[i] = t / R[b][size_t(i) * m + i];
            }
            for (int i = 0; i < k; ++i) yh[size_t(b) * m + i] = {y[i].real(), y[i].imag()};
        }
        HM_HIP(hipMemcpyAsync(K.Y, yh.data(), sizeof(cplx<double>) * nrhs * m, hipMemcpyHostToDevice, s));
        if (mg_status st = set_active(in_cycle)) return st;
        int kmax = 0;
        for (int b = 0; b < nrhs; ++b)
            if (in_cycle[b]) kmax = std::max(kmax, kdir[b]);
        launch_kry_update(lc, g0, K.Z, K.vstride, kmax, K.Y, m, K.X, pl);
        if (mg_status st = check_launch(c)) return st;
        for (int b = 0; b < nrhs; ++b)
            if (stopped[b]) state[b] = 1;
    }
    // final true residuals of every right-hand side
    for (int b = 0; b < nrhs; ++b) c->h_active[b] = 1;
    HM_HIP(hipMemcpyAsync(c->active, c->h_active, sizeof(int) * nrhs, hipMemcpyHostToDevice, s));
    launch_resnorm<double>(lc, op0, vec<double>(K.X, l0), vec<double>(K.F, l0), c->norms);
    lc.active = nullptr;
    launch_copy_out<double>(lc, g0, vec<double>(K.X, l0), x, false, false, false);
    if (mg_status st = check_launch(c)) return st;
    HM_HIP(hipMemcpyAsync(c->h_norms, c->norms, sizeof(RhsNorms) * nrhs, hipMemcpyDeviceToHost, s));
    HM_HIP(hipStreamSynchronize(s));
    mg_status res = MG_OK;
    for (int b = 0; b < nrhs; ++b) {
        rel[b] = nf[b] > 0.0 ? std::sqrt(c->h_norms[b].r2) / nf[b] : 0.0;
        if (state[b] != 1) res = MG_NOT_CONVERGED;
    }
    if (stats) {
        for (int b = 0; b < nrhs; ++b) {
            if (stats->cycles) stats->cycles[b] = its[b];
            if (stats->relres) stats->relres[b] = rel[b];
        }
        if (stats->history) {
            int itmax = 0;
            for (int b = 0; b < nrhs; ++b) itmax = std::max(itmax, its[b]);
            for (int b = 0; b < nrhs; ++b)
                for (int it = its[b]; it < itmax && it < o.max_cycles; ++it) stats->history[size_t(it) * nrhs + b] = NAN;
        }
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return res;
}

}  // extern "C"

namespace {

// Launch settings the autotuner chooses among.
struct TuneSettings {
    int block_cap, tail_n, product, tall_rows, small_rows;
    double ms;
};

void apply_settings(mg_ctx* c, const TuneSettings& t) {
    c->block_cap = t.block_cap;
    c->tail_n = t.tail_n;
    pick_tail_levels(c, t.tail_n);
    c->product_l1 = t.product;
    c->tall_rows = t.tall_rows;
    c->small_rows = t.small_rows;
    clear_graphs(c);
}

// Key of a tuned configuration: the problem shape, the cycle and the device.
std::string tune_key(const mg_ctx* c, int nrhs, int cyc, int smoother, const mg_solve_opts& o) {
    std::string arch = "unknown";
    hipDeviceProp_t prop;
    if (c->device >= 0 && hipGetDeviceProperties(&prop, c->device) == hipSuccess) arch = prop.gcnArchName;
    char buf[512];
    std::snprintf(buf, sizeof(buf), "n=%d levels=%d transfer=%d nrhs=%d cycle=%d smoother=%d nu=%d,%d fp32=%d arch=%s",
                  c->n, c->L, c->transfer, nrhs, cyc, smoother, o.nu_pre, o.nu_post,
                  o.precision == MG_FP32_REFINED ? 1 : 0, arch.c_str());
    return buf;
}

// The cache file holds {"entries": [ {"key": "...", "block_cap": ..., "tail_n": ...,
// "level1_product": ..., "tall_rows": ..., "small_rows": ..., "ms_per_cycle": ...}, ... ]};
// the reader below accepts exactly what tune_cache_write produces (one entry
// per line).
struct CacheEntry {
    std::string key;
    TuneSettings t;
};

bool json_number(const std::string& line, const char* field, double* out) {
    const std::string tag = std::string("\"") + field + "\":";
    const size_t p = line.find(tag);
    if (p == std::string::npos) return false;
    char* end = nullptr;
    const double v = std::strtod(line.c_str() + p + tag.size(), &end);
    if (end == line.c_str() + p + tag.size()) return false;
    *out = v;
    return true;
}

std::vector<CacheEntry> tune_cache_read(const std::string& path) {
    std::vector<CacheEntry> out;
    FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
    std::fclose(f);
    size_t pos = 0;
    while (pos < text.size()) {
        size_t eol = text.find('\n', pos);
        if (eol == std::string::npos) eol = text.size();
        const std::string line = text.substr(pos, eol - pos);
        pos = eol + 1;
        const size_t kp = line.find("\"key\": \"");
        if (kp == std::string::npos) continue;
        const size_t ks = kp + 8, ke = line.find('"', ks);
        if (ke == std::string::npos) continue;
        CacheEntry e;
        e.key = line.substr(ks, ke - ks);
        double v[6];
        if (!json_number(line, "block_cap", &v[0]) || !json_number(line, "tail_n", &v[1]) ||
            !json_number(line, "level1_product", &v[2]) || !json_number(line, "tall_rows", &v[3]) ||
            !json_number(line, "small_rows", &v[4]) || !json_number(line, "ms_per_cycle", &v[5]))
            continue;
        e.t = TuneSettings{int(v[0]), int(v[1]), int(v[2]), int(v[3]), int(v[4]), v[5]};
        out.push_back(e);
    }
    return out;
}

bool tune_cache_write(const std::string& path, const std::vector<CacheEntry>& entries) {
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\"entries\": [\n");
    for (size_t i = 0; i < entries.size(); ++i) {
        const TuneSettings& t = entries[i].t;
        std::fprintf(f,
                     "  {\"key\": \"%s\", \"block_cap\": %d, \"tail_n\": %d, \"level1_product\": %d, "
                     "\"tall_rows\": %d, \"small_rows\": %d, \"ms_per_cycle\": %.6f}%s\n",
                     entries[i].key.c_str(), t.block_cap, t.tail_n, t.product, t.tall_rows, t.small_rows, t.ms,
                     i + 1 < entries.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace

extern "C" {

mg_status mg_tune(mg_handle c, const void* rhs, int nrhs, int cyc, int smoother, const mg_solve_opts* opts,
                  mg_tune_result* out, void* stream) {
    if (!c) return MG_E_ARG;
    const mg_solve_opts o = opts ? *opts : default_solve_opts();
    if (mg_status st = check_solve_args(c, nrhs, 1.0, cyc, smoother, o)) return st;
    if (!is_dev_ptr_ok(rhs)) { c->err = "rhs NULL or misaligned"; return MG_E_ARG; }
    if (c->timing_class != 0) { c->err = "mg_tune needs the timing hook off"; return MG_E_STATE; }
    const std::string key = tune_key(c, nrhs, cyc, smoother, o);
    std::vector<CacheEntry> cache;
    if (!c->tune_cache.empty()) {
        cache = tune_cache_read(c->tune_cache);
        for (const CacheEntry& e : cache)
            if (e.key == key) {
                apply_settings(c, e.t);
                if (out) {
                    *out = mg_tune_result{e.t.block_cap, e.t.tail_n, e.t.product, e.t.ms, 0, e.t.tall_rows,
                                          e.t.small_rows, 1};
                }
                return MG_OK;
            }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    LevelBuf& l0 = c->lv[0];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HM_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        c->err = "hipEventCreate failed";
        return MG_E_HIP;
    }
    struct Guard {
        hipEvent_t a, b;
        ~Guard() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    // launch settings: block cap, tail size, level-1 operator, and the tile
    // shape (block heights on large and on small grids); the heights only
    // matter where such grids exist
    std::vector<int> caps = {320, 640, 1280};
    if (c->max_batch > 1) caps = {64, 160, 320, 640};
    const int tails[] = {0, 16, 32};
    const int prods[] = {0, 1};
    const bool has_tall = c->n >= 256, has_small = (c->n >> 1) <= 128 || c->L > 2;
    std::vector<int> talls = has_tall ? std::vector<int>{4, 8} : std::vector<int>{c->tall_rows};
    std::vector<int> smalls = has_small ? std::vector<int>{2, 4} : std::vector<int>{c->small_rows};
    TuneSettings best{c->block_cap, c->tail_n, c->product_l1, c->tall_rows, c->small_rows, 1e300};
    int tried = 0;
    constexpr int kTimed = 3;
    for (int cap : caps)
        for (int tail : tails)
            for (int prod : prods)
                for (int tr : talls)
                    for (int sr : smalls) {
                        const TuneSettings cand{cap, tail, prod, tr, sr, 0.0};
                        apply_settings(c, cand);
                        LaunchCtx lc = launch_ctx(c, s, nrhs);
                        lc.active = nullptr;
                        launch_copy_in<double>(lc, l0.g, rhs, false, vec<double>(l0.f64, l0), true, false);
                        launch_zero<double>(s, l0.u64, l0.g.plane * nrhs);
                        if (mg_status st = check_launch(c)) return st;
                        SolveRun run(c, nrhs, 1e-300, cyc, smoother, o);
                        if (mg_status st = run.start(s)) return st;
                        HM_HIP(hipStreamSynchronize(s));
                        if (mg_status st = run.begin(s)) return st;
                        auto body = [&](hipStream_t st) { run.enqueue_cycle(st); };
                        if (mg_status st = run_cycle_graph(c, s, run.key, body)) return st;  // warm-up and capture
                        HM_HIP(hipEventRecord(e0, s));
                        for (int k = 0; k < kTimed; ++k)
                            if (mg_status st = run_cycle_graph(c, s, run.key, body)) return st;
                        HM_HIP(hipEventRecord(e1, s));
                        HM_HIP(hipEventSynchronize(e1));
                        float ms = 0.0f;
                        HM_HIP(hipEventElapsedTime(&ms, e0, e1));
                        ++tried;
                        const double per = double(ms) / kTimed;
                        if (per < best.ms) {
                            best = cand;
                            best.ms = per;
                        }
                    }
    apply_settings(c, best);
    HM_HIP(hipStreamSynchronize(s));
    if (!c->tune_cache.empty()) {
        std::vector<CacheEntry> kept;
        for (const CacheEntry& e : cache)
            if (e.key != key) kept.push_back(e);
        kept.push_back(CacheEntry{key, best});
        if (!tune_cache_write(c->tune_cache, kept)) {
            c->err = "mg_tune: could not write the tuning cache " + c->tune_cache;
            return MG_E_ARG;
        }
    }
    if (out) *out = mg_tune_result{best.block_cap, best.tail_n, best.product, best.ms, tried, best.tall_rows,
                                   best.small_rows, 0};
    return MG_OK;
}

mg_status mg_grad(mg_handle c, const void* u, const void* grad_u, int nsrc, double tol, int cyc, int smoother,
                  const mg_solve_opts* opts, double* grad_k2, void* grad_rhs, mg_solve_stats* stats, void* stream) {
    if (!c) return MG_E_ARG;
    const mg_solve_opts o = opts ? *opts : default_solve_opts();
    if (mg_status st = check_solve_args(c, nsrc, tol, cyc, smoother, o)) return st;
    if (mg_status st = check_stats(c, stats, nsrc, o.max_cycles)) return st;
    if (!is_dev_ptr_ok(u) || !is_dev_ptr_ok(grad_u) || !is_dev_ptr_ok(grad_k2)) {
        c->err = "u / grad_u / grad_k2 NULL or misaligned";
        return MG_E_ARG;
    }
    if (grad_rhs && !is_dev_ptr_ok(grad_rhs)) { c->err = "grad_rhs misaligned"; return MG_E_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    LevelBuf& l0 = c->lv[0];
    LaunchCtx lc = launch_ctx(c, s, nsrc);
    lc.active = nullptr;
    // A_s^H lambda = g  <=>  A_s mu = conj(g), lambda = conj(mu)  (A_s complex symmetric)
    launch_copy_in<double>(lc, l0.g, grad_u, false, vec<double>(l0.f64, l0), false, true);
    launch_zero<double>(s, l0.u64, l0.g.plane * nsrc);
    if (mg_status st = check_launch(c)) return st;
    const mg_status res = solve_core(c, s, nsrc, tol, cyc, smoother, o, stats);
    if (res == MG_E_HIP || res == MG_E_ARG) return res;
    // forward solutions into the (idle) level-0 Arnoldi planes
    launch_copy_in<double>(lc, l0.g, u, false, vec<double>(l0.V64, l0), false, false);
    launch_grad_k2(lc, l0.g, c->h, c->k2_64, vec<double>(l0.V64, l0), vec<double>(l0.u64, l0), grad_k2);
    if (grad_rhs) launch_copy_out<double>(lc, l0.g, vec<double>(l0.u64, l0), grad_rhs, false, true, true);
    if (mg_status st = check_launch(c)) return st;
    HM_HIP(hipStreamSynchronize(s));
    return res;
}

mg_status mg_destroy(mg_handle c) {
    if (!c) return MG_OK;
    destroy_pairs(c->ev_pending);
    for (auto& g : c->graphs) {
        destroy_pairs(g.timed);
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    }
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->h_norms) (void)hipHostFree(c->h_norms);
    if (c->h_active) (void)hipHostFree(c->h_active);
    if (c->h_limits) (void)hipHostFree(c->h_limits);
    if (c->h_ring) (void)hipHostFree(c->h_ring);
    if (c->h_hcol) (void)hipHostFree(c->h_hcol);
    for (hipEvent_t e : c->cycle_done)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->hcol_done)
        if (e) (void)hipEventDestroy(e);
    delete c;
    return MG_OK;
}

const char* mg_status_string(mg_status s) {
    switch (s) {
        case MG_OK: return "MG_OK";
        case MG_NOT_CONVERGED: return "MG_NOT_CONVERGED";
        case MG_E_ARG: return "MG_E_ARG";
        case MG_E_HIP: return "MG_E_HIP";
        case MG_E_DIVERGED: return "MG_E_DIVERGED";
        case MG_E_WORKSPACE: return "MG_E_WORKSPACE";
        case MG_E_STATE: return "MG_E_STATE";
    }
    return "unknown status";
}

const char* mg_last_error(mg_handle c) { return c ? c->err.c_str() : g_setup_error.c_str(); }

mg_status mg_level_info(mg_handle c, int level, int* n_l, int* radius, int* levels) {
    if (!c) return MG_E_ARG;
    if (levels) *levels = c->L;
    if (level < 0 || level >= c->L) { c->err = "level out of range"; return MG_E_ARG; }
    if (n_l) *n_l = c->lv[level].g.n;
    if (radius) *radius = c->lv[level].radius;
    return MG_OK;
}

mg_status mg_get_stencil(mg_handle c, int level, void* out, void* stream) {
    if (!c) return MG_E_ARG;
    if (level < 1 || level >= c->L) { c->err = "stencils exist on levels 1 .. L-1"; return MG_E_ARG; }
    if (!is_dev_ptr_ok(out)) { c->err = "out NULL or misaligned"; return MG_E_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const LevelBuf& lb = c->lv[level];
    launch_stencil_out(s, lb.g, lb.radius, lb.coef64, out);
    if (mg_status st = check_launch(c)) return st;
    HM_HIP(hipStreamSynchronize(s));
    return MG_OK;
}

}  // extern "C"

// Level operations run on the level's own buffers: inputs are copied in, the
// step runs, outputs are copied out.
namespace {
template <typename T>
mg_status level_op_run(mg_ctx* c, int kind, int level, const void* a, const void* b, void* out, int nvec,
                       int smoother, int nsteps, double omega, hipStream_t s) {
    LevelBuf& lb = c->lv[level];
    const bool f32 = sizeof(T) == 4;
    LaunchCtx lc = launch_ctx(c, s, nvec);
    lc.active = nullptr;
    auto V = [&](cplx<T>* p) { return vec<T>(p, lb); };
    cplx<T>* U = Prec<T>::u(lb);
    cplx<T>* F = Prec<T>::f(lb);
    cplx<T>* Wv = Prec<T>::w(lb);
    switch (kind) {
        case 0:  // apply
            launch_copy_in<T>(lc, lb.g, a, f32, V(U), false, false);
            launch_apply<T>(lc, level_op<T>(c, level), V(U), V(Wv));
            launch_copy_out<T>(lc, lb.g, V(Wv), out, f32, false, false);
            break;
        case 1:  // residual
            launch_copy_in<T>(lc, lb.g, a, f32, V(U), false, false);
            launch_copy_in<T>(lc, lb.g, b, f32, V(F), false, false);
            launch_residual<T>(lc, level_op<T>(c, level), V(U), V(F), V(Wv));
            launch_copy_out<T>(lc, lb.g, V(Wv), out, f32, false, false);
            break;
        case 2: {  // smooth
            launch_copy_in<T>(lc, lb.g, out, f32, V(U), false, false);
            launch_copy_in<T>(lc, lb.g, b, f32, V(F), false, false);
            for (int i = 0; i < nvec; ++i) c->h_active[i] = 1;
            HM_HIP(hipMemcpyAsync(c->active, c->h_active, sizeof(int) * nvec, hipMemcpyHostToDevice, s));
            lc.active = c->active;
            const CycleParams cp{1, smoother, 0, 0, omega};
            const int saved = c->cur_buf;
            for (int k = 0; k < nsteps;) {
                const int js = smoother == MG_JACOBI && k + 1 < nsteps ? 2 : 1;
                smooth<T>(c, lc, level, cp, false, 0, ProlongIn<T>{}, false, nullptr, js);
                k += js;
            }
            c->cur_buf = saved;
            launch_copy_out<T>(lc, lb.g, V(Prec<T>::u(lb)), out, f32, false, false);
            break;
        }
        case 3: {  // restrict
            LevelBuf& cb = c->lv[level + 1];
            launch_copy_in<T>(lc, lb.g, a, f32, V(Wv), false, false);
            launch_restrict<T>(lc, lb.g, cb.g, c->transfer, V(Wv), vec<T>(Prec<T>::f(cb), cb), Vec<T>{nullptr, 0});
            launch_copy_out<T>(lc, cb.g, vec<T>(Prec<T>::f(cb), cb), out, f32, false, false);
            break;
        }
        case 4: {  // prolong-add
            LevelBuf& cb = c->lv[level + 1];
            launch_copy_in<T>(lc, cb.g, a, f32, vec<T>(Prec<T>::u(cb), cb), false, false);
            launch_copy_in<T>(lc, lb.g, out, f32, V(U), false, false);
            launch_prolong_add<T>(lc, cb.g, lb.g, c->transfer, vec<T>(Prec<T>::u(cb), cb), V(U));
            launch_copy_out<T>(lc, lb.g, V(U), out, f32, false, false);
            break;
        }
        case 5: {  // coarsest solve
            launch_copy_in<T>(lc, lb.g, a, f32, V(F), false, false);
            launch_coarse_solve<T>(lc, lb.g, c->dense, c->piv, V(F), V(U));
            launch_copy_out<T>(lc, lb.g, V(U), out, f32, false, false);
            break;
        }
    }
    if (mg_status st = check_launch(c)) return st;
    HM_HIP(hipStreamSynchronize(s));
    return MG_OK;
}

// r = f - A_l x with x, f and r staged through the static device scratch
// (nvec planes each, x's planes zeroed first so that its ghost frame reads
// zero): the kernels of mg_residual, enqueued only.
template <typename T>
mg_status residual_static(mg_ctx* c, int level, const void* x, const void* f, void* r, int nvec, char* scr,
                          hipStream_t s) {
    const LevelBuf& lb = c->lv[level];
    const bool f32 = sizeof(T) == 4;
    const size_t pbytes = align_up(size_t(lb.g.plane) * sizeof(cplx<T>) * size_t(nvec), kAlign);
    cplx<T>* X = reinterpret_cast<cplx<T>*>(scr);
    cplx<T>* F = reinterpret_cast<cplx<T>*>(scr + pbytes);
    cplx<T>* Rr = reinterpret_cast<cplx<T>*>(scr + 2 * pbytes);
    LaunchCtx lc = launch_ctx(c, s, nvec);
    lc.active = nullptr;
    launch_fill_words(s, X, (long long)pbytes, 0u);
    launch_copy_in<T>(lc, lb.g, x, f32, vec<T>(X, lb), false, false);
    launch_copy_in<T>(lc, lb.g, f, f32, vec<T>(F, lb), false, false);
    launch_residual<T>(lc, level_op<T>(c, level), vec<T>(X, lb), vec<T>(F, lb), vec<T>(Rr, lb));
    launch_copy_out<T>(lc, lb.g, vec<T>(Rr, lb), r, f32, false, false);
    return check_launch(c);
}

mg_status level_entry(mg_ctx* c, int kind, int level, const void* a, const void* b, void* out, int nvec,
                      int precision, int smoother, int nsteps, double omega, void* stream) {
    if (nvec < 1 || nvec > c->max_batch) { c->err = "nvec must be in [1, max_batch]"; return MG_E_ARG; }
    if (precision == MG_FP64)
        return level_op_run<double>(c, kind, level, a, b, out, nvec, smoother, nsteps, omega,
                                    static_cast<hipStream_t>(stream));
    return level_op_run<float>(c, kind, level, a, b, out, nvec, smoother, nsteps, omega,
                               static_cast<hipStream_t>(stream));
}
}  // namespace

extern "C" {

mg_status mg_apply(mg_handle c, int level, const void* x, void* y, int nvec, int precision, void* stream) {
    if (!c) return MG_E_ARG;
    if (mg_status st = check_level(c, level, precision, true)) return st;
    if (!is_dev_ptr_ok(x) || !is_dev_ptr_ok(y)) { c->err = "NULL or misaligned vector"; return MG_E_ARG; }
    return level_entry(c, 0, level, x, nullptr, y, nvec, precision, 0, 0, 0.0, stream);
}

mg_status mg_residual(mg_handle c, int level, const void* x, const void* f, void* r, int nvec, int precision,
                      void* stream) {
    if (!c) return MG_E_ARG;
    if (mg_status st = check_level(c, level, precision, true)) return st;
    if (!is_dev_ptr_ok(x) || !is_dev_ptr_ok(f) || !is_dev_ptr_ok(r)) { c->err = "NULL or misaligned vector"; return MG_E_ARG; }
    return level_entry(c, 1, level, x, f, r, nvec, precision, 0, 0, 0.0, stream);
}

mg_status mg_residual_noalloc(mg_handle c, int level, const void* x, const void* f, void* r, int nvec, int precision,
                              void* stream) {
    if (!c) return MG_E_ARG;
    if (mg_status st = check_level(c, level, precision, true)) return st;
    if (!is_dev_ptr_ok(x) || !is_dev_ptr_ok(f) || !is_dev_ptr_ok(r)) { c->err = "NULL or misaligned vector"; return MG_E_ARG; }
    if (nvec < 1) { c->err = "nvec must be >= 1"; return MG_E_ARG; }
    const size_t elem = precision == MG_FP64 ? 16 : 8;
    const size_t need = 3 * align_up(size_t(c->lv[level].g.plane) * elem * size_t(nvec), kAlign);
    if (need > kStaticScratchBytes) {
        c->err = "mg_residual_noalloc: 3 x nvec padded planes of level " + std::to_string(level) + " need " +
                 std::to_string(need) + " bytes, beyond the " + std::to_string(kStaticScratchBytes) +
                 "-byte static scratch";
        return MG_E_ARG;
    }
    int dev = -1;
    HM_HIP(hipGetDevice(&dev));
    if (dev != c->device) {
        c->err = "mg_residual_noalloc: the handle's device (set up on " + std::to_string(c->device) +
                 ") must be current";
        return MG_E_ARG;
    }
    void* scr = nullptr;
    HM_HIP(static_scratch(dev, &scr));
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(scr);
    if (precision == MG_FP64) return residual_static<double>(c, level, x, f, r, nvec, base, s);
    return residual_static<float>(c, level, x, f, r, nvec, base, s);
}

mg_status mg_smooth(mg_handle c, int level, int smoother, int nsteps, double omega, void* u, const void* f, int nvec,
                    int precision, void* stream) {
    if (!c) return MG_E_ARG;
    if (mg_status st = check_level(c, level, precision, true)) return st;
    if (smoother != MG_JACOBI && smoother != MG_GMRES3) { c->err = "unknown smoother"; return MG_E_ARG; }
    if (nsteps < 0 || !(omega > 0.0)) { c->err = "nsteps >= 0 and omega > 0 required"; return MG_E_ARG; }
    if (!is_dev_ptr_ok(u) || !is_dev_ptr_ok(f)) { c->err = "NULL or misaligned vector"; return MG_E_ARG; }
    return level_entry(c, 2, level, nullptr, f, u, nvec, precision, smoother, nsteps, omega, stream);
}

mg_status mg_restrict(mg_handle c, int level, const void* fine, void* coarse, int nvec, int precision, void* stream) {
    if (!c) return MG_E_ARG;
    if (mg_status st = check_level(c, level, precision, false)) return st;
    if (!is_dev_ptr_ok(fine) || !is_dev_ptr_ok(coarse)) { c->err = "NULL or misaligned vector"; return MG_E_ARG; }
    return level_entry(c, 3, level, fine, nullptr, coarse, nvec, precision, 0, 0, 0.0, stream);
}

mg_status mg_prolong_add(mg_handle c, int level, const void* coarse, void* fine, int nvec, int precision,
                         void* stream) {
    if (!c) return MG_E_ARG;
    if (mg_status st = check_level(c, level, precision, false)) return st;
    if (!is_dev_ptr_ok(fine) || !is_dev_ptr_ok(coarse)) { c->err = "NULL or misaligned vector"; return MG_E_ARG; }
    return level_entry(c, 4, level, coarse, nullptr, fine, nvec, precision, 0, 0, 0.0, stream);
}

mg_status mg_coarse_solve(mg_handle c, const void* f, void* u, int nvec, int precision, void* stream) {
    if (!c) return MG_E_ARG;
    if (mg_status st = check_level(c, c->L - 1, precision, true)) return st;
    if (!is_dev_ptr_ok(f) || !is_dev_ptr_ok(u)) { c->err = "NULL or misaligned vector"; return MG_E_ARG; }
    return level_entry(c, 5, c->L - 1, f, nullptr, u, nvec, precision, 0, 0, 0.0, stream);
}

mg_status mg_cycle(mg_handle c, void* u, const void* f_s, int nvec, int cyc, int smoother, const mg_solve_opts* opts,
                   void* stream) {
    if (!c) return MG_E_ARG;
    const mg_solve_opts o = opts ? *opts : default_solve_opts();
    if (mg_status st = check_solve_args(c, nvec, 1.0, cyc, smoother, o)) return st;
    const bool f32 = o.precision == MG_FP32_REFINED;
    if (f32 && !c->has32) { c->err = "FP32 cycle needs a setup with FP32 data"; return MG_E_ARG; }
    if (!is_dev_ptr_ok(u) || !is_dev_ptr_ok(f_s)) { c->err = "NULL or misaligned vector"; return MG_E_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    LevelBuf& l0 = c->lv[0];
    LaunchCtx lc = launch_ctx(c, s, nvec);
    lc.active = nullptr;
    if (f32) {
        launch_copy_in<float>(lc, l0.g, f_s, true, vec<float>(l0.f32, l0), false, false);
        launch_copy_in<float>(lc, l0.g, u, true, vec<float>(l0.u32, l0), false, false);
    } else {
        launch_copy_in<double>(lc, l0.g, f_s, false, vec<double>(l0.f64, l0), false, false);
        launch_copy_in<double>(lc, l0.g, u, false, vec<double>(l0.u64, l0), false, false);
    }
    for (int i = 0; i < nvec; ++i) c->h_active[i] = 1;
    HM_HIP(hipMemcpyAsync(c->active, c->h_active, sizeof(int) * nvec, hipMemcpyHostToDevice, s));
    lc.active = c->active;
    const CycleParams cp{cyc, smoother, o.nu_pre, o.nu_post, o.omega};
    if (f32) {
        cycle<float>(c, lc, 0, cp);
        launch_copy_out<float>(lc, l0.g, vec<float>(l0.u32, l0), u, true, false, false);
    } else {
        cycle<double>(c, lc, 0, cp);
        launch_copy_out<double>(lc, l0.g, vec<double>(l0.u64, l0), u, false, false, false);
    }
    if (mg_status st = check_launch(c)) return st;
    HM_HIP(hipStreamSynchronize(s));
    return MG_OK;
}

mg_status mg_set_timing(mg_handle c, int kernel_class) {
    if (!c) return MG_E_ARG;
    if (kernel_class < 0 || kernel_class > 4) { c->err = "unknown kernel class"; return MG_E_ARG; }
    c->timing_class = kernel_class;
    destroy_pairs(c->ev_pending);
    c->last_graph = -1;
    c->t_launches = 0;
    c->t_ms = 0.0;
    c->t_nodes = 0.0;
    return MG_OK;
}

mg_status mg_get_timing(mg_handle c, int* launches, double* total_ms, double* nodes_per_launch) {
    if (!c) return MG_E_ARG;
    harvest_timing(c);
    if (launches) *launches = c->t_launches;
    if (total_ms) *total_ms = c->t_ms;
    if (nodes_per_launch) *nodes_per_launch = c->t_launches ? c->t_nodes / c->t_launches : 0.0;
    return MG_OK;
}

}  // extern "C"
