// C ABI of the library and the host-side schedule of the full multigrid pass.
//
// Per MLMC level l (Algorithm 3 of the paper), for a device-resident batch of
// samples:
//   1. KL synthesis (matrix cores) -> injected coefficient pyramid;
//   2. correction-operator pyramids (face averaging) for the two QoI stages
//      and the FP64 inverses of the coarsest operators;
//   3. full multigrid: direct solve on the coarsest grid, then for each finer
//      grid an interpolated start and cycles - one per intermediate stage, and
//      until ||b - A p|| <= tol ||b|| on the stages n_l/2 (gives Q^c_l) and n_l
//      (gives Q^f_l). Converged samples drop out of every later launch through
//      a per-sample activity mask.
//   FP32_IR: cycles in FP32; on the QoI stages FP64 iterative refinement
//   (p64 += e32, r = b - A64 p64) decides convergence and yields the QoI.
//
// Scheduling: after the first cycle of a QoI stage, cycles run in blocks of G
// (cycle + convergence check each); the host reads the number of samples still
// iterating once per block. A block can be captured once into a HIP graph and
// replayed. Several MLMC levels can run at once, each on its own stream and
// workspace (fmgmc_solve_levels). G, graph use and the batch size per level
// come from a measured autotuner (fmgmc_autotune). None of these choices
// changes any result: the same kernels run on the same samples in the same order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "cnn.h"
#include "common.h"

namespace fmgmc {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

namespace {

constexpr int kMaxGrid = 9;    // grid indices: n_coarsest << k
constexpr int kSmallTop = 32;  // grids up to this size run whole cycles in LDS
constexpr int kMaxLanes = 16;  // most concurrent levels in fmgmc_solve_levels (one hardware queue each)

int ilog2(int v) {
    int r = 0;
    while ((1 << (r + 1)) <= v) ++r;
    return r;
}

bool is_device_ptr(const void *p) {
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

template <typename T>
int dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) return FMGMC_OK;
    if (hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc failed (" + std::to_string(count * sizeof(T)) + " bytes)");
        return FMGMC_ENOMEM;
    }
    return FMGMC_OK;
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

template <typename T>
struct Pyr {
    Faces<T> f[kMaxGrid];
};

#define TRY(x)                           \
    do {                                 \
        int rc_ = (x);                   \
        if (rc_ != FMGMC_OK) return rc_; \
    } while (0)

// Schedule parameters of one MLMC level (never change results).
struct Tune {
    int check_every = 1;   // cycles per host read of the active count
    int graphs = 0;        // replay the cycle block from a captured HIP graph
    int batch = 0;         // samples per device chunk (0 = workspace capacity)
};

// Device buffers for a batch of up to S_max samples of one hierarchy.
struct Work {
    int S_max = 0;
    int ng = 0;                       // grid levels 0..ng-1
    int nsz[kMaxGrid] = {};
    double *K64[kMaxGrid] = {};
    float *K32[kMaxGrid] = {};
    double *x64[kMaxGrid] = {}, *b64[kMaxGrid] = {}, *p64[kMaxGrid] = {};
    float *x32[kMaxGrid] = {}, *b32[kMaxGrid] = {};
    Pyr<double> pf64[2];
    Pyr<float> pf32[2];
    double *chol = nullptr;  // [3][S][N0*N0]: inverses of stage op, coarse-stage pyramid, fine-stage pyramid
    double *rr = nullptr, *q = nullptr, *bnorm = nullptr, *qf = nullptr, *qc = nullptr, *xi = nullptr;
    unsigned char *klx = nullptr;  // xi in matrix-core operand order (FP32 / BF16 KL contraction)
    int32_t *active = nullptr, *cycles = nullptr, *n_active = nullptr;
    uint8_t *flags = nullptr;
    int32_t *h_n_active = nullptr;  // pinned, 2 slots (cycle blocks in flight)
    hipEvent_t blk_ev[2] = {};      // the copy of each in-flight block's active count
    int n_active_host = 0;
    int top_grid = -1;
    bool profile = false;           // profiling records allowed for this workspace
    hipStream_t own_stream = nullptr;
    // learned warm start: inference activations (bf16, act_cap bytes each), residual
    // norms at the FMG start, and for training pairs the FMG start itself
    void *act[2] = {};
    size_t act_cap = 0;
    double *rr0 = nullptr;
    double *p0 = nullptr;
    size_t p0_cap = 0;
    float *capx_base[2] = {}, *capt_base[2] = {};  // training-pair outputs (slot 0 coarse, 1 fine)
    float *cap_x[2] = {}, *cap_t[2] = {};          // the current chunk's views
    // captured cycle blocks, keyed by (MLMC level, stage grid, block length, batch size)
    std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;
};

void free_work(Work &w) {
    for (int k = 0; k < kMaxGrid; ++k) {
        dfree(w.K64[k]); dfree(w.K32[k]); dfree(w.x64[k]); dfree(w.b64[k]); dfree(w.p64[k]);
        dfree(w.x32[k]); dfree(w.b32[k]);
        for (int q = 0; q < 2; ++q) {
            dfree(w.pf64[q].f[k].fx); dfree(w.pf64[q].f[k].fy); dfree(w.pf64[q].f[k].fxe);
            dfree(w.pf64[q].f[k].fyn);
            dfree(w.pf32[q].f[k].fx); dfree(w.pf32[q].f[k].fy); dfree(w.pf32[q].f[k].fxe);
            dfree(w.pf32[q].f[k].fyn);
        }
    }
    dfree(w.chol); dfree(w.rr); dfree(w.q); dfree(w.bnorm); dfree(w.qf); dfree(w.qc); dfree(w.xi);
    dfree(w.klx);
    dfree(w.active); dfree(w.cycles); dfree(w.n_active); dfree(w.flags);
    for (int k = 0; k < 2; ++k)
        if (w.act[k]) (void)hipFree(w.act[k]);
    w.act[0] = w.act[1] = nullptr;
    w.act_cap = 0;
    dfree(w.rr0); dfree(w.p0);
    w.p0_cap = 0;
    if (w.h_n_active) (void)hipHostFree(w.h_n_active);
    w.h_n_active = nullptr;
    for (auto &e : w.blk_ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    for (auto &kv : w.graphs) (void)hipGraphExecDestroy(kv.second);
    w.graphs.clear();
    if (w.own_stream) (void)hipStreamDestroy(w.own_stream);
    w.own_stream = nullptr;
}

}  // namespace
}  // namespace fmgmc

using namespace fmgmc;

struct fmgmc_ctx {
    fmgmc_field field;
    fmgmc_hier hier;
    fmgmc_opts opts;
    int device = 0;
    ModeTable table;
    int small_top = 0;   // largest grid index handled by the LDS kernel
    // constants
    std::vector<double *> d_phi;  // per MLMC level [kmax+1][n_l]
    int32_t *d_ma = nullptr, *d_mb = nullptr;
    double *d_sqrtlam = nullptr;
    Work main;                                  // finest-level workspace (fmgmc_solve_level)
    std::vector<std::unique_ptr<Work>> lev;     // per-level workspaces (fmgmc_solve_levels)
    std::vector<hipStream_t> lanes;             // fmgmc_solve_levels: one stream per host thread
    std::vector<Tune> tune;                     // per MLMC level
    const fmgmc_cnn *warm = nullptr;            // learned warm start
    int warm_min_n = 256;
    int warm_max_n = 0;                         // 0: no upper bound
    fmgmc_cnn *owned_warm = nullptr;            // network loaded from opts.cnn_weights (owned)
    std::string tune_path;                      // opts.tune_cache ("" = none)
    // measurement hooks
    struct Rec {
        hipEvent_t a, b;
        double alg;
    };
    bool prof = false;
    std::vector<Rec> prof_rec[FMGMC_PROF_KINDS];
    // FP32_IR: FP64 context (same field, hierarchy and stopping rule) that
    // re-solves the samples the mixed-precision form leaves unconverged;
    // created on first use, shared by the per-level threads under fb_mu
    fmgmc_ctx *fallback = nullptr;
    std::mutex fb_mu;
};

namespace {

bool ir_mode(const fmgmc_ctx *c) { return c->opts.solver == FMGMC_SOLVER_FP32_IR; }

Bnd bnd(const fmgmc_ctx *c) {
    const fmgmc_hier &h = c->hier;
    return Bnd{h.p_west, h.p_east, h.p_south, h.p_north, h.boundary == FMGMC_BC_DIRICHLET ? 1 : 0};
}

template <typename T>
int alloc_faces(Faces<T> &f, int S, int n) {
    TRY(dalloc(&f.fx, size_t(S) * n * n));
    TRY(dalloc(&f.fy, size_t(S) * n * n));
    TRY(dalloc(&f.fxe, size_t(S) * n));
    TRY(dalloc(&f.fyn, size_t(S) * n));
    return FMGMC_OK;
}

// Workspace for S samples of a hierarchy whose finest grid is n_top.
int alloc_work(const fmgmc_ctx *c, Work &w, int S, int n_top) {
    const int M = c->table.M;
    const bool ir = ir_mode(c);
    w.S_max = S;
    w.ng = ilog2(n_top / c->hier.n_coarsest) + 1;
    for (int k = 0; k < w.ng; ++k) w.nsz[k] = c->hier.n_coarsest << k;
    const int t = w.ng - 1;
    for (int k = 0; k <= t; ++k) {
        const size_t N = size_t(S) * w.nsz[k] * w.nsz[k];
        if (!ir) {
            TRY(dalloc(&w.K64[k], N));
            TRY(dalloc(&w.x64[k], N));
            TRY(dalloc(&w.b64[k], N));
        } else {
            TRY(dalloc(&w.K32[k], N));
            TRY(dalloc(&w.x32[k], N));
            TRY(dalloc(&w.b32[k], N));
            if (k >= 1) {  // FP64 operator and iterate only where a QoI stage can sit
                TRY(dalloc(&w.K64[k], N));
                TRY(dalloc(&w.p64[k], N));
            }
        }
        if (k < t) {
            for (int q = 0; q < 2; ++q) {
                if (q == 0 && k >= t - 1) continue;  // coarse-stage pyramid stops below n_l / 2
                if (!ir) TRY(alloc_faces(w.pf64[q].f[k], S, w.nsz[k]));
                else TRY(alloc_faces(w.pf32[q].f[k], S, w.nsz[k]));
            }
        }
    }
    const int N0 = w.nsz[0] * w.nsz[0];
    TRY(dalloc(&w.chol, size_t(3) * S * N0 * N0));
    TRY(dalloc(&w.rr, S)); TRY(dalloc(&w.q, S)); TRY(dalloc(&w.bnorm, S));
    TRY(dalloc(&w.qf, S)); TRY(dalloc(&w.qc, S)); TRY(dalloc(&w.xi, size_t(S) * M));
    TRY(dalloc(&w.klx, kl_work_bytes(S, M, c->opts.kl_prec)));
    TRY(dalloc(&w.active, S)); TRY(dalloc(&w.cycles, 2 * size_t(S))); TRY(dalloc(&w.n_active, 1));
    TRY(dalloc(&w.flags, S));
    TRY(dalloc(&w.rr0, S));
    if (hipHostMalloc(reinterpret_cast<void **>(&w.h_n_active), 2 * sizeof(int32_t)) != hipSuccess) {
        set_error("hipHostMalloc failed");
        return FMGMC_ENOMEM;
    }
    for (auto &e : w.blk_ev) FMGMC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return FMGMC_OK;
}

int alloc_constants(fmgmc_ctx *c) {
    const int M = c->table.M;
    const int nk = c->table.kmax + 1;
    TRY(dalloc(&c->d_ma, M)); TRY(dalloc(&c->d_mb, M)); TRY(dalloc(&c->d_sqrtlam, M));
    std::vector<double> sl(M);
    for (int m = 0; m < M; ++m) sl[m] = std::sqrt(c->table.lam[m]);
    FMGMC_HIP(hipMemcpy(c->d_ma, c->table.a.data(), M * sizeof(int32_t), hipMemcpyHostToDevice));
    FMGMC_HIP(hipMemcpy(c->d_mb, c->table.b.data(), M * sizeof(int32_t), hipMemcpyHostToDevice));
    FMGMC_HIP(hipMemcpy(c->d_sqrtlam, sl.data(), M * sizeof(double), hipMemcpyHostToDevice));
    c->d_phi.assign(c->hier.n_levels, nullptr);
    for (int l = 0; l < c->hier.n_levels; ++l) {
        const int n = c->hier.n0 << l;
        std::vector<double> tab;
        tabulate_phi(c->table, n, tab);
        TRY(dalloc(&c->d_phi[l], size_t(nk) * n));
        FMGMC_HIP(hipMemcpy(c->d_phi[l], tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    return FMGMC_OK;
}

void free_ctx(fmgmc_ctx *c) {
    if (c->owned_warm) {
        fmgmc_cnn_destroy(c->owned_warm);
        c->owned_warm = nullptr;
    }
    if (c->fallback) {
        fmgmc_destroy(c->fallback);
        c->fallback = nullptr;
    }
    for (auto &p : c->d_phi) dfree(p);
    c->d_phi.clear();
    dfree(c->d_ma); dfree(c->d_mb); dfree(c->d_sqrtlam);
    free_work(c->main);
    for (auto &w : c->lev)
        if (w) free_work(*w);
    c->lev.clear();
    for (auto &st : c->lanes)
        if (st) (void)hipStreamDestroy(st);
    c->lanes.clear();
}

// ------------------------------------------------------------ measurement
// Brackets one launch with events when profiling is on (never inside a capture).
template <typename F>
int timed(fmgmc_ctx *c, Work &w, int kind, double alg, hipStream_t st, F &&launch) {
    if (!c->prof || !w.profile) return launch();
    fmgmc_ctx::Rec r{nullptr, nullptr, alg};
    FMGMC_HIP(hipEventCreate(&r.a));
    FMGMC_HIP(hipEventCreate(&r.b));
    FMGMC_HIP(hipEventRecord(r.a, st));
    const int rc = launch();
    FMGMC_HIP(hipEventRecord(r.b, st));
    c->prof_rec[kind].push_back(r);
    return rc;
}

// ------------------------------------------------------------------ cycles
template <typename T>
struct Bufs {
    T **K, **x, **b;
    Pyr<T> *pf;
};

Bufs<double> bufs64(Work &w) { return {w.K64, w.x64, w.b64, w.pf64}; }
Bufs<float> bufs32(Work &w) { return {w.K32, w.x32, w.b32, w.pf32}; }

// How a cycle's top-grid passes join its neighbours (FP32 cycles back to back):
// VC_SKIP_PRE, the previous cycle's last pass already did this cycle's
// pre-smoothing and restriction; VC_FUSE_POST, the post-smoothing pass also
// does the next cycle's pre-smoothing and restriction.
template <typename T>
int pyramid(fmgmc_ctx *c, Work &W, Bufs<T> B, int S, int q, int top, bool from_k, hipStream_t st);

enum { VC_SKIP_PRE = 1, VC_FUSE_POST = 2, VC_TOP_FACES = 4 };
// VC_TOP_FACES (the FP64 form's top stage, level >= 1): its first pre-smoothing
// pass also writes the faces on n/2 of the stage's correction pyramid (skipped by
// prepare), which is then finished before the coarse-grid correction.

// One cycle with top grid k: top operator from K (stage operator), the levels
// below from correction pyramid q; V(nu1,nu2) on grids above w_max_n, two
// coarse cycles (W) on grids n <= w_max_n. rhs_array: top rhs in b[k] (else the
// Dirichlet data). init: INIT_ZERO / INIT_LOAD / INIT_INTERP (from x[k-1]).
// flow (VC_*) only for a top grid above small_top, in FP32 with rhs_array.
template <typename T>
int vcycle(fmgmc_ctx *c, Work &W, Bufs<T> B, int S, int k, int q, int init, bool rhs_array, int out_top,
           hipStream_t st, int flow = 0) {
    const int nh1 = 2 * c->opts.nu1, nh2 = 2 * c->opts.nu2;
    const int N0 = W.nsz[0] * W.nsz[0];
    const Bnd g = bnd(c);
    const double *chol_pyr = W.chol + size_t(1 + q) * S * N0 * N0;
    const double *chol_stage = W.chol;
    auto gamma = [&](int j) { return (j > 0 && W.nsz[j] <= c->opts.w_max_n) ? 2 : 1; };
    auto small = [&](int top, bool from_k, int sinit, bool srhs, int sout, const double *chol) {
        SmallArgs<T> a{};
        a.top = top;
        for (int j = 0; j <= top; ++j) a.ns[j] = W.nsz[j];
        a.top_from_k = from_k;
        a.Ktop = B.K[top];
        for (int j = 0; j < 8; ++j) a.f[j] = B.pf[q].f[j];
        a.chol = chol;
        a.x = B.x[top];
        a.b = B.b[top];
        a.xc = top > 0 ? B.x[top - 1] : nullptr;
        a.rr = W.rr;
        a.q = W.q;
        a.active = W.active;
        a.g = g;
        a.nu1 = c->opts.nu1;
        a.nu2 = c->opts.nu2;
        a.wmax = c->opts.w_max_n;
        return launch_small(a, S, sinit, srhs, sout, st);
    };
    if (k <= c->small_top) {
        // whole cycle in LDS (k == 0: the direct solve with the stage operator)
        return small(k, true, init, rhs_array, out_top, k == 0 ? chol_stage : chol_pyr);
    }
    auto march = [&](int j, bool ck, int minit, bool rhsa, int mout, int nh) {
        MarchArgs<T> a{};
        a.n = W.nsz[j];
        a.x = B.x[j];
        a.b = B.b[j];
        a.K = B.K[j];
        a.f = (mout & OUT_FACES) ? B.pf[1].f[j - 1] : B.pf[q].f[j];
        a.xc = B.x[j - 1];
        a.bc = B.b[j - 1];
        a.rr = W.rr;
        a.q = W.q;
        a.active = W.active;
        a.g = g;
        return launch_march(a, S, nh, ck, minit, rhsa, mout, st);
    };
    // cycle rooted at correction level j (rhs b[j], faces of pyramid q)
    std::function<int(int, int)> corr = [&](int j, int cinit) -> int {
        if (j <= c->small_top) return small(j, false, cinit, true, 0, chol_pyr);
        TRY(march(j, false, cinit, true, OUT_RESTRICT, nh1));
        for (int g = 0; g < gamma(j - 1); ++g) TRY(corr(j - 1, g == 0 ? INIT_ZERO : INIT_LOAD));
        return march(j, false, INIT_PROLONG, true, 0, nh2);
    };
    // algorithmic bytes per cell of the top-grid passes (each operand once)
    const double w = sizeof(T), cells = double(W.nsz[k]) * W.nsz[k];
    const bool top = (k == W.top_grid);
    const double act = double(W.n_active_host);
    const double b_pre = (init == INIT_ZERO ? 0.0 : (init == INIT_INTERP ? 0.25 * w : w)) + w /*K*/ +
                         (rhs_array ? w : 0.0) + w /*x out*/ + 0.25 * w /*restricted residual*/;
    const double b_post = w + 0.25 * w + w + (rhs_array ? w : 0.0) + w;
    if (!(flow & VC_SKIP_PRE)) {
        const int out_pre = OUT_RESTRICT | ((flow & VC_TOP_FACES) ? OUT_FACES : 0);
        // (the faces: west and south on n/2, a quarter of the cells each)
        const double b_faces = (flow & VC_TOP_FACES) ? 0.5 * w : 0.0;
        if (top) TRY(timed(c, W, FMGMC_PROF_PRE, act * cells * (b_pre + b_faces), st, [&] { return march(k, true, init, rhs_array, out_pre, nh1); }));
        else TRY(march(k, true, init, rhs_array, out_pre, nh1));
        if (flow & VC_TOP_FACES) TRY(pyramid<T>(c, W, B, S, 1, k, false, st));
    }
    for (int g = 0; g < gamma(k - 1); ++g) TRY(corr(k - 1, g == 0 ? INIT_ZERO : INIT_LOAD));
    if (flow & VC_FUSE_POST) {
        // x, coarse correction, K, b in; x and the restricted residual out
        const double b_fused = w + 0.25 * w + w + w + w + 0.25 * w;
        if (top) TRY(timed(c, W, FMGMC_PROF_FUSED, act * cells * b_fused, st, [&] { return march(k, true, INIT_PROLONG, true, OUT_RESTRICT, nh2 + nh1); }));
        else TRY(march(k, true, INIT_PROLONG, true, OUT_RESTRICT, nh2 + nh1));
        return FMGMC_OK;
    }
    if (top) TRY(timed(c, W, FMGMC_PROF_POST, act * cells * b_post, st, [&] { return march(k, true, INIT_PROLONG, rhs_array, out_top, nh2); }));
    else TRY(march(k, true, INIT_PROLONG, rhs_array, out_top, nh2));
    return FMGMC_OK;
}

int read_active(Work &W, hipStream_t st, int *out) {
    FMGMC_HIP(hipMemcpyAsync(W.h_n_active, W.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FMGMC_HIP(hipStreamSynchronize(st));
    *out = *W.h_n_active;
    W.n_active_host = *out;
    return FMGMC_OK;
}

int launch_checks(fmgmc_ctx *c, Work &W, int S, int slot, double *qout, int inc, double tol, hipStream_t st) {
    CheckArgs a{};
    a.rr = W.rr;
    a.bnorm = W.bnorm;
    a.q = W.q;
    a.active = W.active;
    a.cycles = W.cycles;
    a.slot = slot;
    a.inc = inc;
    a.flags = W.flags;
    a.qout = qout;
    a.tol = tol;
    a.max_cycles = c->opts.max_cycles;
    a.n_active = W.n_active;
    return launch_check(a, S, st);
}

// Runs `block` (G cycles + checks) eagerly or from a captured graph. The graph
// is captured on its first use for a (level, stage grid, block length, batch
// size) key and replayed afterwards; it holds kernel launches only, whose
// arguments are workspace addresses and per-context constants.
int run_block(Work &W, bool use_graph, std::tuple<int, int, int, int> key, hipStream_t st,
              const std::function<int()> &block) {
    if (!use_graph || st == nullptr) return block();  // no capture on the null stream
    auto it = W.graphs.find(key);
    if (it == W.graphs.end()) {
        hipGraph_t g = nullptr;
        FMGMC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const int rc = block();
        const hipError_t e = hipStreamEndCapture(st, &g);
        if (rc != FMGMC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) {
            set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            return FMGMC_EHIP;
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
            return FMGMC_EHIP;
        }
        it = W.graphs.emplace(key, ex).first;
    }
    FMGMC_HIP(hipGraphLaunch(it->second, st));
    return FMGMC_OK;
}

// Correction pyramid q of the QoI stage `top`: its faces on n_top/2 from K
// (unless a pass over the stage grid has written them), coarsened level by
// level, and the inverse of its coarsest operator.
template <typename T>
int pyramid(fmgmc_ctx *c, Work &W, Bufs<T> B, int S, int q, int top, bool from_k, hipStream_t st) {
    const int all = bnd(c).all;
    const int N0 = W.nsz[0] * W.nsz[0];
    if (from_k) TRY(launch_faces_from_k<T>(W.nsz[top], B.K[top], all, B.pf[q].f[top - 1], S, st));
    for (int j = top - 1; j >= 1; --j)
        TRY(launch_faces_coarsen<T>(W.nsz[j], B.pf[q].f[j], B.pf[q].f[j - 1], S, st));
    return launch_chol<T>(W.nsz[0], nullptr, B.pf[q].f[0], false, all, W.chol + size_t(1 + q) * S * N0 * N0, S,
                          st);
}

// Build correction pyramids and coarsest inverses for a batch. With skip_top,
// the pyramid of the level's top stage (q = 1, used by that stage only when
// level >= 1) is left to the stage itself: its first refinement pass writes the
// faces on n_top/2 (fmgmc::pyramid then runs from there).
template <typename T>
int prepare(fmgmc_ctx *c, Work &W, Bufs<T> B, int S, int level, int t, hipStream_t st, bool skip_top = false) {
    const int all = bnd(c).all;
    Faces<T> none{};
    TRY(launch_chol<T>(W.nsz[0], B.K[0], none, true, all, W.chol, S, st));
    for (int q = 0; q < 2; ++q) {
        const int top = (q == 1) ? t : t - 1;  // QoI stage that owns the pyramid
        if (q == 0 && level == 0) continue;
        if (top < 1) continue;
        if (q == 1 && skip_top) continue;
        TRY(pyramid<T>(c, W, B, S, q, top, true, st));
    }
    return FMGMC_OK;
}

// Cycles of one QoI stage after its first step (first_done cycles): blocks of G
// steps of per_cycle cycles (+ check), until no sample is left or max_cycles is
// reached. Each block ends with an asynchronous copy of the number of samples
// still iterating, and the next block is enqueued before that count reaches the
// host, so the device never waits for the host between blocks. A block
// enqueued after every sample has converged is a set of empty launches (each
// kernel returns at once for an inactive sample), so the results are those of
// one block at a time. With profiling on, blocks run one at a time: the
// recorded traffic counts the samples active at each launch.
int iterate_stage(fmgmc_ctx *c, Work &W, const Tune &tn, int level, int k, int S, int first_done, int per_cycle,
                  int na, hipStream_t st, const std::function<int()> &cycle_and_check) {
    const int G = std::max(1, tn.check_every);
    const bool prof = c->prof && W.profile;
    const int ahead = prof ? 1 : 2;  // blocks whose count the host has not read yet
    int done = first_done, inflight = 0, next = 0;
    int slots[2] = {0, 0};
    if (na < 0) {  // the first step's count is not read yet: it is the first block in flight
        FMGMC_HIP(hipMemcpyAsync(W.h_n_active, W.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        FMGMC_HIP(hipEventRecord(W.blk_ev[0], st));
        slots[inflight++] = 0;
        next = 1;
        na = 1;
    }
    while (true) {
        if (na > 0 && done < c->opts.max_cycles && inflight < ahead) {
            const int g = std::min(G, (c->opts.max_cycles - done + per_cycle - 1) / per_cycle);
            // only full chunks are captured: a ragged chunk runs eagerly, so arbitrary
            // sample counts (the adaptive drivers' increments) add no graphs and the
            // cache holds at most one per (level, stage grid, block length)
            const int full = (tn.batch > 0 && tn.batch < W.S_max) ? tn.batch : W.S_max;
            const bool graph = tn.graphs && !prof && S == full;
            TRY(run_block(W, graph, std::make_tuple(level, k, g, S), st, [&]() -> int {
                for (int i = 0; i < g; ++i) TRY(cycle_and_check());
                return FMGMC_OK;
            }));
            const int slot = next;
            next ^= 1;
            FMGMC_HIP(hipMemcpyAsync(W.h_n_active + slot, W.n_active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            FMGMC_HIP(hipEventRecord(W.blk_ev[slot], st));
            slots[inflight++] = slot;
            done += g * per_cycle;
            continue;
        }
        if (inflight == 0) break;
        const int slot = slots[0];
        FMGMC_HIP(hipEventSynchronize(W.blk_ev[slot]));
        na = W.h_n_active[slot];
        W.n_active_host = na;
        slots[0] = slots[1];
        --inflight;
    }
    return FMGMC_OK;
}

// FMG-MLMC (default): one pass whose stages n_l/2 and n_l both run to the
// tolerance, giving Q^c_l and Q^f_l (Section 2.5, Algorithm 3). With
// separate_coarse (the standard-MLMC comparator, levels >= 1): Q^c_l from its own
// FMG pass ending at n_l/2, then a pass to n_l in which n_l/2 is an ordinary
// intermediate stage (one cycle). Both passes use the injected coefficients.
template <typename P>
int run_passes(fmgmc_ctx *c, int level, int t, double *qf, double *qc, P &&pass) {
    if (level >= 1 && c->opts.separate_coarse) {
        TRY(pass(t - 1, false, qc, 0));
        return pass(t, false, qf, 1);
    }
    return pass(t, level >= 1, qf, 1);
}

int run_batch_fp64(fmgmc_ctx *c, Work &W, const Tune &tn, int level, int S, double *qf, double *qc,
                   hipStream_t st) {
    const int t = ilog2((c->hier.n0 << level) / W.nsz[0]);
    Bufs<double> B = bufs64(W);
    // the top stage's first pass writes the faces on n/2 of its pyramid (pyramid 1
    // serves only the top stage when level >= 1)
    const bool top_faces = level >= 1 && t > c->small_top;
    TRY(prepare<double>(c, W, B, S, level, t, st, top_faces));
    const double tol = c->opts.rel_tol;
    // one FMG pass up to stage ktop; with_coarse: stage ktop - 1 is a QoI stage too
    auto pass = [&](int ktop, bool with_coarse, double *qtop, int slot_top) -> int {
        for (int k = 0; k <= ktop; ++k) {
            const bool fine = (k == ktop), coarse = (with_coarse && k == ktop - 1);
            const int q = (level >= 1 && k <= t - 1) ? 0 : 1;
            TRY(launch_fill_i32(W.active, 1, S, st));
            W.n_active_host = S;
            if (!(fine || coarse)) {
                TRY(vcycle<double>(c, W, B, S, k, q, k == 0 ? INIT_ZERO : INIT_INTERP, false, 0, st));
                continue;
            }
            double *qout = fine ? qtop : qc;
            const int slot = fine ? slot_top : 0;
            TRY(launch_bnorm<double>(W.nsz[k], B.K[k], bnd(c), W.bnorm, S, st));
            int na;
            if (k == 0) {  // direct solve: exact, no cycles
                TRY(vcycle<double>(c, W, B, S, 0, q, INIT_ZERO, false, OUT_RR | OUT_Q, st));
                TRY(launch_checks(c, W, S, slot, qout, 0, INFINITY, st));
                TRY(read_active(W, st, &na));
                continue;
            }
            TRY(vcycle<double>(c, W, B, S, k, q, INIT_INTERP, false, OUT_RR | OUT_Q, st,
                               (top_faces && k == t) ? VC_TOP_FACES : 0));
            TRY(launch_checks(c, W, S, slot, qout, 1, tol, st));
            TRY(iterate_stage(c, W, tn, level, k, S, 1, 1, -1, st, [&]() -> int {
                TRY(vcycle<double>(c, W, B, S, k, q, INIT_LOAD, false, OUT_RR | OUT_Q, st));
                return launch_checks(c, W, S, slot, qout, 1, tol, st);
            }));
        }
        return FMGMC_OK;
    };
    return run_passes(c, level, t, qf, qc, pass);
}

// Learned warm start of one QoI stage (p64 holds the FMG start p~, rr its
// residual norm, r32 its residual): p~ + rms(r) y, then the plain start is
// restored for every sample whose residual did not drop.
template <typename F, typename R>
int warm_start(fmgmc_ctx *c, Work &W, int k, int S, const IRArgs &ia, hipStream_t st, F &&interp, R &&refine) {
    const int n = W.nsz[k];
    InferArgs a{};
    a.n = n;
    a.S = S;
    a.in0 = W.K32[k];
    a.in1 = W.b32[k];
    a.in_stride = int64_t(n) * n;
    a.log0 = 1;
    a.rr = W.rr0;
    a.e = W.x32[k];  // rms(r) y in FP32 (the stage's FP32 iterate is free until its first cycle)
    a.active = W.active;
    // useful flops per cell, 2 per multiply-add: first layer 18 x 32, four residual
    // layers 288 x 32 each, output layer 288
    const double flops = double(W.n_active_host) * n * n * 2.0 * (18.0 * 32 + 4.0 * 288 * 32 + 288);
    // all layers in one pass with the activations on chip
    TRY(timed(c, W, FMGMC_PROF_CNN, flops, st, [&] { return launch_cnn_fused(a, cnn_packed(c->warm), st); }));
    // p += rms(r) y in FP64 and the residual of the corrected start, in one refinement pass
    IRArgs iw = ia;
    iw.e = W.x32[k];
    TRY(refine(iw));
    TRY(launch_judge(S, W.rr, W.rr0, W.active, W.flags, st));  // active <- samples to restore
    TRY(interp());
    TRY(refine(ia));
    return launch_fill_i32(W.active, 1, S, st);
}

int run_batch_ir(fmgmc_ctx *c, Work &W, const Tune &tn, int level, int S, double *qf, double *qc,
                 hipStream_t st) {
    const int t = ilog2((c->hier.n0 << level) / W.nsz[0]);
    Bufs<float> B = bufs32(W);
    // refinement passes fused with the next cycle's pre-smoothing (see the stage
    // loop); then the top stage's first one also writes the faces of its
    // correction pyramid (pyramid 1 serves only the top stage when level >= 1)
    const bool fuse_ir_top = c->opts.fuse_cycles && t > c->small_top && c->opts.nu1 <= 2 &&
                             c->opts.nu1 + c->opts.nu2 <= 4;
    const bool top_faces = fuse_ir_top && level >= 1;
    TRY(prepare<float>(c, W, B, S, level, t, st, top_faces));
    const double tol = c->opts.rel_tol;
    const Bnd g = bnd(c);
    // one FMG pass up to stage ktop; with_coarse: stage ktop - 1 is a QoI stage too
    auto pass = [&](int ktop, bool with_coarse, double *qtop, int slot_top) -> int {
        for (int k = 0; k <= ktop; ++k) {
            const bool fine = (k == ktop), coarse = (with_coarse && k == ktop - 1);
            const int q = (level >= 1 && k <= t - 1) ? 0 : 1;
            TRY(launch_fill_i32(W.active, 1, S, st));
            W.n_active_host = S;
            if (!(fine || coarse)) {
                TRY(vcycle<float>(c, W, B, S, k, q, k == 0 ? INIT_ZERO : INIT_INTERP, false, 0, st));
                continue;
            }
            double *qout = fine ? qtop : qc;
            const int slot = fine ? slot_top : 0;
            const int n = W.nsz[k];
            // FMG start in FP64: from the FP64 solution when the stage below was a QoI stage
            auto interp = [&]() -> int {
                if (fine && with_coarse) return launch_interp64<double>(n, W.p64[k - 1], W.p64[k], W.active, g, S, st);
                return launch_interp64<float>(n, W.x32[k - 1], W.p64[k], W.active, g, S, st);
            };
            // back-to-back cycles on a marching top grid share their joining pass
            const bool fuse = c->opts.fuse_cycles && k > c->small_top && c->opts.nu1 + c->opts.nu2 <= 4;
            // ... and every refinement also does the pre-smoothing and restriction of
            // the FP32 cycle after it (which then skips its own): the refinement's
            // residual is that cycle's right-hand side, and its coefficients are
            // float(K64), the stage's FP32 K
            const bool fuse_ir = fuse && c->opts.nu1 <= 2;
            const bool warm = c->warm && n >= c->warm_min_n && (c->warm_max_n == 0 || n <= c->warm_max_n);
            // the faces of the top stage's pyramid (skipped by prepare) come from its
            // first refinement pass, which also forms the FMG start from the FP64
            // solution below it (the separate interpolation pass is then not run)
            const bool faces_here = top_faces && k == t;
            const bool pin = faces_here && fuse_ir && !warm && fine && with_coarse;
            if (!pin) TRY(interp());
            TRY(launch_bnorm<double>(n, W.K64[k], g, W.bnorm, S, st));
            IRArgs ia{};
            ia.n = n;
            ia.p = W.p64[k];
            ia.e = nullptr;
            ia.K = W.K64[k];
            ia.r32 = W.b32[k];
            ia.rr = W.rr;
            ia.q = W.q;
            ia.active = W.active;
            ia.g = g;
            // refinement pass: p (+= e), r = b - A p in FP64, r -> FP32, ||r||^2, Q
            auto refine = [&](const IRArgs &a, bool faces = false, bool pstart = false) -> int {
                const double cells = double(W.n_active_host) * double(n) * n;
                if (!fuse_ir) {
                    // reads p, e and K, writes p and r (without e: reads p and K, writes r)
                    const double b = cells * (a.e ? 8.0 + 4.0 + 8.0 + 8.0 + 4.0 : 8.0 + 8.0 + 4.0);
                    if (k == W.top_grid) return timed(c, W, FMGMC_PROF_IR, b, st, [&] { return launch_ir(a, S, st); });
                    return launch_ir(a, S, st);
                }
                MarchArgs<float> m{};
                m.n = n;
                m.x = W.x32[k];
                m.bc = W.b32[k - 1];
                m.rr = a.rr;
                m.q = a.q;
                m.active = a.active;
                m.g = a.g;
                m.p = a.p;
                m.e = a.e;
                m.K64 = a.K;
                m.r32 = a.r32;
                if (faces) m.f = B.pf[1].f[k - 1];
                if (pstart) m.pc = W.p64[k - 1];
                const int out = OUT_RESTRICT | (a.e ? OUT_PUPD : 0) | (faces ? OUT_FACES : 0) |
                                (pstart ? OUT_PINTERP : 0);
                // the refinement's bytes, then x and the restricted residual out (and
                // the west and south faces on n/2; with the start formed in the pass, p
                // is written instead of read and the solution on n/2 read)
                const double b = cells * ((a.e ? 8.0 + 4.0 + 8.0 + 8.0 + 4.0 : 8.0 + 8.0 + 4.0) + 4.0 + 1.0 +
                                          (faces ? 2.0 : 0.0) + (pstart ? 2.0 : 0.0));
                auto go = [&] { return launch_march(m, S, 2 * c->opts.nu1, true, INIT_IR, true, out, st); };
                if (k == W.top_grid) return timed(c, W, FMGMC_PROF_IRPRE, b, st, go);
                return go();
            };
            // first residual of the stage (with the warm start, the network's input:
            // a plain refinement pass, the warm start's own passes then do the rest)
            if (warm && fuse_ir) {
                const double irb0 = double(W.n_active_host) * double(n) * n * (8.0 + 8.0 + 4.0);
                if (k == W.top_grid) TRY(timed(c, W, FMGMC_PROF_IR, irb0, st, [&] { return launch_ir(ia, S, st); }));
                else TRY(launch_ir(ia, S, st));
                if (faces_here) TRY(pyramid<float>(c, W, B, S, 1, t, true, st));
            } else {
                TRY(refine(ia, faces_here, pin));
                if (faces_here) TRY(pyramid<float>(c, W, B, S, 1, t, false, st));
            }
            float *capx = W.cap_x[slot], *capt = W.cap_t[slot];
            if (warm || capx) TRY(launch_copy_f64(W.rr, W.rr0, S, st));
            if (capx) {
                TRY(launch_pack_x(n, S, W.K32[k], W.b32[k], W.rr0, capx, st));
                TRY(launch_copy_f64(W.p64[k], W.p0, int64_t(S) * n * n, st));
            }
            if (warm) TRY(warm_start(c, W, k, S, ia, st, interp, refine));
            // FP32 cycles before the first FP64 refinement, and per refinement after it
            const int inner = std::max(1, c->opts.inner_cycles);
            const int first = std::min(c->opts.inner_first > 0 ? c->opts.inner_first : inner, c->opts.max_cycles);
            auto step = [&](int ni) -> int {
                for (int ic = 0; ic < ni; ++ic) {
                    const int flow = fuse ? (((ic > 0 || fuse_ir) ? VC_SKIP_PRE : 0) | (ic + 1 < ni ? VC_FUSE_POST : 0)) : 0;
                    TRY(vcycle<float>(c, W, B, S, k, q, ic == 0 ? INIT_ZERO : INIT_LOAD, true, 0, st, flow));
                }
                IRArgs iu = ia;
                iu.e = W.x32[k];
                TRY(refine(iu));
                return launch_checks(c, W, S, slot, qout, ni, tol, st);
            };
            TRY(step(first));
            TRY(iterate_stage(c, W, tn, level, k, S, first, inner, -1, st, [&] { return step(inner); }));
            if (capt) TRY(launch_pack_t(n, S, W.p64[k], W.p0, W.rr0, capt, st));
        }
        return FMGMC_OK;
    };
    return run_passes(c, level, t, qf, qc, pass);
}

int validate(const fmgmc_field *f, const fmgmc_hier *h, const fmgmc_opts *o) {
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    if (!f || !h || !o) return FMGMC_EINVAL;
    if (f->cov_kind != FMGMC_COV_SEPARABLE_EXP || !(f->sigma2 > 0) || !(f->corr_len > 0) || f->n_modes < 1 ||
        f->n_modes > 4096)
        return FMGMC_EINVAL;
    if (h->n_levels < 1 || !pow2(h->n0) || h->n_coarsest != 4 || h->n0 < h->n_coarsest) return FMGMC_EINVAL;
    if (h->boundary != FMGMC_BC_MIXED && h->boundary != FMGMC_BC_DIRICHLET) return FMGMC_EINVAL;
    if (!std::isfinite(h->p_west) || !std::isfinite(h->p_east) || !std::isfinite(h->p_south) ||
        !std::isfinite(h->p_north))
        return FMGMC_EINVAL;
    const int nf = h->n0 << (h->n_levels - 1);
    if (nf > 1024) return FMGMC_EINVAL;
    if (o->solver != FMGMC_SOLVER_FP64 && o->solver != FMGMC_SOLVER_FP32_IR) return FMGMC_EINVAL;
    if (o->kl_prec < FMGMC_KL_FP64 || o->kl_prec > FMGMC_KL_FP64_DENSE) return FMGMC_EINVAL;
    // smoothing sweeps: 1..2 in FP64 cycles, 1..4 in FP32 cycles
    const int nu_max = o->solver == FMGMC_SOLVER_FP32_IR ? 4 : 2;
    if (o->nu1 < 1 || o->nu1 > nu_max || o->nu2 < 1 || o->nu2 > nu_max || o->max_cycles < 1 || !(o->rel_tol > 0))
        return FMGMC_EINVAL;
    if (o->solver == FMGMC_SOLVER_FP32_IR && h->n0 < 8) return FMGMC_EINVAL;  // QoI stages need n >= 8
    if (o->max_batch < 0 || o->w_max_n < 0 || o->separate_coarse < 0 || o->separate_coarse > 1) return FMGMC_EINVAL;
    if (o->fuse_cycles < 0 || o->fuse_cycles > 1) return FMGMC_EINVAL;
    if (o->warm != FMGMC_WARM_NONE && o->warm != FMGMC_WARM_CNN) return FMGMC_EINVAL;
    if (o->warm == FMGMC_WARM_CNN &&
        (o->solver != FMGMC_SOLVER_FP32_IR || h->boundary != FMGMC_BC_MIXED || !o->cnn_weights))
        return FMGMC_EINVAL;
    if (o->warm_min_n != 0 && o->warm_min_n < 16) return FMGMC_EINVAL;
    if (o->warm_max_n < 0) return FMGMC_EINVAL;
    return FMGMC_OK;
}

// Schedule file: a header naming the hierarchy and solver it was measured for,
// then one line per tuned level: "level check_every graphs batch".
std::string tune_header(const fmgmc_ctx *c) {
    char b[160];
    std::snprintf(b, sizeof(b), "fmgmc-schedule 1 levels %d n0 %d solver %d boundary %d", c->hier.n_levels,
                  c->hier.n0, c->opts.solver, c->hier.boundary);
    return b;
}

void read_tune_cache(fmgmc_ctx *c) {
    if (c->tune_path.empty()) return;
    std::ifstream f(c->tune_path);
    std::string head;
    if (!f || !std::getline(f, head) || head != tune_header(c)) return;
    int l, G, gr, b;
    while (f >> l >> G >> gr >> b)
        if (l >= 0 && l < c->hier.n_levels && G >= 1 && (gr == 0 || gr == 1) && b >= 0) c->tune[l] = Tune{G, gr, b};
}

int write_tune_cache(const fmgmc_ctx *c) {
    if (c->tune_path.empty()) return FMGMC_OK;
    std::ofstream f(c->tune_path, std::ios::trunc);
    if (!f) {
        set_error("cannot write the schedule file " + c->tune_path);
        return FMGMC_EINVAL;
    }
    f << tune_header(c) << "\n";
    for (int l = 0; l < c->hier.n_levels; ++l)
        f << l << " " << c->tune[l].check_every << " " << c->tune[l].graphs << " " << c->tune[l].batch << "\n";
    return f.good() ? FMGMC_OK : FMGMC_EINVAL;
}

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(d);
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// One MLMC level on workspace W: chunks of at most tn.batch samples.
// FP32_IR samples of a chunk that missed rel_tol within max_cycles (finite
// ones) are solved again by the FP64 FMG pass on the same field; their Q,
// cycles and flags are replaced in the caller's arrays (host or device) and
// FMGMC_FLAG_FP64 is set. hf holds the chunk's flags on the host and is
// updated. xdev: the chunk's coordinates on the device.
int fp64_fallback(fmgmc_ctx *ctx, int level, int S, int64_t s0, const double *xdev, double *q_fine,
                  double *q_coarse, int32_t *cycles, uint8_t *flags, std::vector<uint8_t> &hf) {
    std::vector<int> bad;
    for (int s = 0; s < S; ++s)
        if ((hf[s] & FMGMC_FLAG_NOTCONV) && !(hf[s] & FMGMC_FLAG_NONFINITE)) bad.push_back(s);
    if (bad.empty()) return FMGMC_OK;
    std::lock_guard<std::mutex> lock(ctx->fb_mu);
    if (!ctx->fallback) {
        fmgmc_opts o = ctx->opts;
        o.solver = FMGMC_SOLVER_FP64;
        o.nu1 = std::min(o.nu1, 2);
        o.nu2 = std::min(o.nu2, 2);
        o.max_batch = 64;
        o.fuse_cycles = 0;
        o.warm = FMGMC_WARM_NONE;
        o.cnn_weights = nullptr;
        o.tune_cache = nullptr;
        TRY(fmgmc_create(&ctx->fallback, &ctx->field, &ctx->hier, &o, ctx->device));
    }
    const int M = ctx->table.M, nb = int(bad.size());
    std::vector<double> xb(size_t(nb) * M), qf(nb), qc(nb);
    std::vector<int32_t> cy(2 * size_t(nb));
    std::vector<uint8_t> fl(nb);
    for (int i = 0; i < nb; ++i)
        FMGMC_HIP(hipMemcpy(xb.data() + size_t(i) * M, xdev + size_t(bad[i]) * M, M * sizeof(double),
                            hipMemcpyDeviceToHost));
    const int rc = fmgmc_solve_level(ctx->fallback, level, nb, xb.data(), qf.data(), qc.data(), cy.data(),
                                     fl.data(), nullptr);
    if (rc != FMGMC_OK && rc != FMGMC_ENOTCONV && rc != FMGMC_ENONFINITE) return rc;
    for (int i = 0; i < nb; ++i) {
        const int64_t g = s0 + bad[i];
        hf[bad[i]] = uint8_t(fl[i] | FMGMC_FLAG_FP64 | (hf[bad[i]] & FMGMC_FLAG_WARM_REJECTED));
        FMGMC_HIP(hipMemcpy(q_fine + g, &qf[i], sizeof(double), hipMemcpyDefault));
        FMGMC_HIP(hipMemcpy(q_coarse + g, &qc[i], sizeof(double), hipMemcpyDefault));
        if (cycles) FMGMC_HIP(hipMemcpy(cycles + 2 * g, &cy[2 * size_t(i)], 2 * sizeof(int32_t), hipMemcpyDefault));
        if (flags) FMGMC_HIP(hipMemcpy(flags + g, &hf[bad[i]], 1, hipMemcpyDefault));
    }
    return FMGMC_OK;
}

int solve_level_on(fmgmc_ctx *ctx, Work &W, const Tune &tn, int level, int64_t n_samples, const double *xi,
                   double *q_fine, double *q_coarse, int32_t *cycles, uint8_t *flags, hipStream_t st,
                   bool *any_notconv, bool *any_nonfinite) {
    const int M = ctx->table.M;
    const int n = ctx->hier.n0 << level;
    const int t = ilog2(n / W.nsz[0]);
    const bool ir = ir_mode(ctx);
    const bool xi_dev = is_device_ptr(xi), qf_dev = is_device_ptr(q_fine), qc_dev = is_device_ptr(q_coarse);
    const bool cy_dev = cycles && is_device_ptr(cycles), fl_dev = flags && is_device_ptr(flags);
    const int chunk = (tn.batch > 0 && tn.batch < W.S_max) ? tn.batch : W.S_max;
    std::vector<uint8_t> hflags;
    for (int64_t s0 = 0; s0 < n_samples; s0 += chunk) {
        const int S = int(std::min<int64_t>(chunk, n_samples - s0));
        const double *x = xi + size_t(s0) * M;
        if (!xi_dev) {
            FMGMC_HIP(hipMemcpyAsync(W.xi, x, size_t(S) * M * sizeof(double), hipMemcpyHostToDevice, st));
            x = W.xi;
        }
        // the batch writes Q into the workspace (fixed addresses, so captured
        // cycle blocks stay valid for every chunk and call) and copies it out
        double *qf = W.qf, *qc = W.qc;
        TRY(launch_fill_i32(W.cycles, 0, 2 * int64_t(S), st));
        TRY(launch_fill_u8(W.flags, 0, S, st));
        TRY(launch_fill_f64(qc, 0.0, S, st));
        KLArgs a{};
        a.n = n;
        a.M = M;
        a.xi = x;
        a.phi = ctx->d_phi[level];
        a.kdim = ctx->table.kmax + 1;
        a.ma = ctx->d_ma;
        a.mb = ctx->d_mb;
        a.sqrtlam = ctx->d_sqrtlam;
        a.xw = W.klx;
        a.nlev = t + 1;
        for (int j = 0; j <= t; ++j) {
            const int k = t - j;  // pyramid slot j = grid index t - j
            a.K64[j] = W.K64[k];
            a.K32[j] = ir ? W.K32[k] : nullptr;
            if (ir && !(k == t || (level >= 1 && k == t - 1))) a.K64[j] = nullptr;
        }
        W.top_grid = t;
        for (int sl = 0; sl < 2; ++sl) {
            const int ns = sl == 1 ? n : n / 2;
            W.cap_x[sl] = W.capx_base[sl] ? W.capx_base[sl] + size_t(s0) * 2 * ns * ns : nullptr;
            W.cap_t[sl] = W.capt_base[sl] ? W.capt_base[sl] + size_t(s0) * ns * ns : nullptr;
        }
        const double klf = kl_flops(a, ctx->opts.kl_prec) * S;
        TRY(timed(ctx, W, FMGMC_PROF_KL, klf, st, [&] { return launch_kl(a, S, ctx->opts.kl_prec, st); }));
        TRY(ir ? run_batch_ir(ctx, W, tn, level, S, qf, qc, st) : run_batch_fp64(ctx, W, tn, level, S, qf, qc, st));
        FMGMC_HIP(hipMemcpyAsync(q_fine + s0, qf, S * sizeof(double),
                                 qf_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
        FMGMC_HIP(hipMemcpyAsync(q_coarse + s0, qc, S * sizeof(double),
                                 qc_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
        if (cycles)
            FMGMC_HIP(hipMemcpyAsync(cycles + 2 * s0, W.cycles, 2 * size_t(S) * sizeof(int32_t),
                                     cy_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
        if (flags && fl_dev) FMGMC_HIP(hipMemcpyAsync(flags + s0, W.flags, S, hipMemcpyDeviceToDevice, st));
        hflags.resize(S);
        FMGMC_HIP(hipMemcpyAsync(hflags.data(), W.flags, S, hipMemcpyDeviceToHost, st));
        FMGMC_HIP(hipStreamSynchronize(st));
        if (flags && !fl_dev) std::memcpy(flags + s0, hflags.data(), S);
        if (ir) TRY(fp64_fallback(ctx, level, S, s0, x, q_fine, q_coarse, cycles, flags, hflags));
        for (int s = 0; s < S; ++s) {
            *any_notconv |= (hflags[s] & FMGMC_FLAG_NOTCONV) != 0;
            *any_nonfinite |= (hflags[s] & FMGMC_FLAG_NONFINITE) != 0;
        }
    }
    return FMGMC_OK;
}

int status_of(bool notconv, bool nonfinite, const char *who) {
    if (nonfinite) {
        set_error(std::string(who) + ": non-finite residual in some samples (see flags)");
        return FMGMC_ENONFINITE;
    }
    if (notconv) {
        set_error(std::string(who) + ": some samples did not reach rel_tol (see flags)");
        return FMGMC_ENOTCONV;
    }
    return FMGMC_OK;
}

// Per-level workspace for fmgmc_solve_levels / fmgmc_autotune (created on first
// use): the finest-level workspace's memory budget, at most 16384 samples.
int level_work(fmgmc_ctx *c, int level, Work **out) {
    if (!c->lev[level]) {
        std::unique_ptr<Work> w(new Work());
        const int n = c->hier.n0 << level;
        const double scale = std::pow(double(c->hier.n0 << (c->hier.n_levels - 1)) / n, 2.0);
        const int S = int(std::min<double>(16384.0, std::max<double>(c->main.S_max, c->main.S_max * scale)));
        int rc = alloc_work(c, *w, S, n);
        if (rc == FMGMC_OK && hipStreamCreateWithFlags(&w->own_stream, hipStreamNonBlocking) != hipSuccess) {
            set_error("hipStreamCreate failed");
            rc = FMGMC_EHIP;
        }
        if (rc != FMGMC_OK) {
            free_work(*w);
            return rc;
        }
        c->lev[level] = std::move(w);
    }
    *out = c->lev[level].get();
    return FMGMC_OK;
}

// Combines the per-level results of the estimator reduction (h: mean_y, var_y,
// mean_qf, var_qf, mean_qc) into the level records and the MLMC sum (Eq. (5))
// with its variance; the sum over the levels is compensated (Neumaier).
struct EstAcc {
    double total = 0.0, totc = 0.0, var = 0.0;
    void add(int l, int64_t n, int n_shifts, const double *h, fmgmc_level_est *levels) {
        if (levels) {
            levels[l].n = n;
            levels[l].mean_y = h[0];
            levels[l].var_y = h[1];
            levels[l].mean_qf = h[2];
            levels[l].var_qf = h[3];
            levels[l].mean_qc = h[4];
        }
        const double tt = total + h[0];
        totc += (std::fabs(total) >= std::fabs(h[0])) ? (total - tt) + h[0] : (h[0] - tt) + total;
        total = tt;
        var += (n_shifts > 1) ? h[1] : h[1] / double(n);
    }
    void finish(double *mean, double *var_of_mean) const {
        if (mean) *mean = total + totc;
        if (var_of_mean) *var_of_mean = var;
    }
};

}  // namespace

extern "C" {

const char *fmgmc_last_error(void) { return g_err.c_str(); }

int fmgmc_version(void) { return 10100; }

int fmgmc_create(fmgmc_ctx **out, const fmgmc_field *field, const fmgmc_hier *hier, const fmgmc_opts *opts,
                 int device) {
    if (!out) {
        set_error("fmgmc_create: out is NULL");
        return FMGMC_EINVAL;
    }
    *out = nullptr;
    if (validate(field, hier, opts) != FMGMC_OK) {
        set_error("fmgmc_create: invalid field / hierarchy / options");
        return FMGMC_EINVAL;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        set_error("fmgmc_create: no such HIP device");
        return FMGMC_EHIP;
    }
    DevGuard g(device);
    std::unique_ptr<fmgmc_ctx> c(new fmgmc_ctx());
    c->field = *field;
    c->hier = *hier;
    c->opts = *opts;
    c->device = device;
    if (c->opts.inner_cycles < 1) c->opts.inner_cycles = 1;
    if (c->opts.inner_first < 0) c->opts.inner_first = 0;
    if (opts->tune_cache) c->tune_path = opts->tune_cache;
    c->opts.tune_cache = nullptr;  // no caller pointer is kept
    c->opts.cnn_weights = nullptr;
    int rc = build_mode_table(field->sigma2, field->corr_len, field->n_modes, c->table);
    if (rc != FMGMC_OK) {
        set_error("fmgmc_create: mode table");
        return rc;
    }
    const int nf = hier->n0 << (hier->n_levels - 1);
    if (ilog2(nf / hier->n_coarsest) + 1 > kMaxGrid) {
        set_error("fmgmc_create: too many grid levels");
        return FMGMC_EINVAL;
    }
    c->small_top = ilog2(kSmallTop / hier->n_coarsest);
    c->lev.resize(hier->n_levels);
    c->tune.assign(hier->n_levels, Tune());
    c->main.profile = true;
    rc = alloc_constants(c.get());
    if (rc == FMGMC_OK) rc = alloc_work(c.get(), c->main, opts->max_batch > 0 ? opts->max_batch : 1024, nf);
    if (rc == FMGMC_OK && opts->warm == FMGMC_WARM_CNN) {
        rc = fmgmc_cnn_create(&c->owned_warm, 0, device);
        if (rc == FMGMC_OK) rc = fmgmc_cnn_load(c->owned_warm, opts->cnn_weights);
        if (rc == FMGMC_OK)
            rc = fmgmc_set_warm_range(c.get(), c->owned_warm, opts->warm_min_n > 0 ? opts->warm_min_n : 256,
                                      opts->warm_max_n);
    }
    if (rc != FMGMC_OK) {
        free_ctx(c.get());
        return rc;
    }
    read_tune_cache(c.get());
    *out = c.release();
    return FMGMC_OK;
}

int fmgmc_kl_modes(double sigma2, double corr_len, int32_t n_modes, int32_t *a, int32_t *b, double *lambda) {
    ModeTable t;
    const int rc = build_mode_table(sigma2, corr_len, n_modes, t);
    if (rc != FMGMC_OK) {
        set_error("fmgmc_kl_modes: invalid field");
        return rc;
    }
    for (int m = 0; m < t.M; ++m) {
        if (a) a[m] = t.a[m];
        if (b) b[m] = t.b[m];
        if (lambda) lambda[m] = t.lam[m];
    }
    return FMGMC_OK;
}

int fmgmc_profile_enable(fmgmc_ctx *ctx, int32_t enable) {
    if (!ctx) return FMGMC_EINVAL;
    ctx->prof = enable != 0;
    return FMGMC_OK;
}

int fmgmc_profile_read(fmgmc_ctx *ctx, int32_t kind, double *ms, int64_t *launches, double *alg) {
    if (!ctx || kind < 0 || kind >= FMGMC_PROF_KINDS) {
        set_error("fmgmc_profile_read: bad arguments");
        return FMGMC_EINVAL;
    }
    DevGuard g(ctx->device);
    double tot = 0.0, bytes = 0.0;
    int64_t cnt = 0;
    int rc = FMGMC_OK;
    for (auto &r : ctx->prof_rec[kind]) {
        float t = 0.f;
        if (rc == FMGMC_OK &&
            (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)) {
            set_error("fmgmc_profile_read: event error");
            rc = FMGMC_EHIP;
        }
        tot += t;
        bytes += r.alg;
        ++cnt;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    ctx->prof_rec[kind].clear();
    if (ms) *ms = tot;
    if (launches) *launches = cnt;
    if (alg) *alg = bytes;
    return rc;
}

int fmgmc_destroy(fmgmc_ctx *ctx) {
    if (!ctx) return FMGMC_OK;
    DevGuard g(ctx->device);
    for (int k = 0; k < FMGMC_PROF_KINDS; ++k) {
        int64_t n;
        fmgmc_profile_read(ctx, k, nullptr, &n, nullptr);
    }
    free_ctx(ctx);
    delete ctx;
    return FMGMC_OK;
}

int fmgmc_mode_table(const fmgmc_ctx *ctx, int32_t *a, int32_t *b, double *lambda, int32_t cap) {
    if (!ctx || cap < 0) {
        set_error("fmgmc_mode_table: bad arguments");
        return FMGMC_EINVAL;
    }
    const int m = std::min<int>(cap, ctx->table.M);
    for (int k = 0; k < m; ++k) {
        if (a) a[k] = ctx->table.a[k];
        if (b) b[k] = ctx->table.b[k];
        if (lambda) lambda[k] = ctx->table.lam[k];
    }
    return m;
}

int fmgmc_synthesize_field(fmgmc_ctx *ctx, int32_t level, int64_t n_samples, const double *xi, double *k_out,
                           void *stream) {
    if (!ctx || level < 0 || level >= ctx->hier.n_levels || n_samples < 0 || (n_samples > 0 && (!xi || !k_out))) {
        set_error("fmgmc_synthesize_field: bad arguments");
        return FMGMC_EINVAL;
    }
    DevGuard g(ctx->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int n = ctx->hier.n0 << level, M = ctx->table.M;
    const bool xi_dev = is_device_ptr(xi), k_dev = is_device_ptr(k_out);
    double *tmp = nullptr;
    const int chunk = ctx->main.S_max;
    if (!k_dev) TRY(dalloc(&tmp, size_t(chunk) * n * n));
    int rc = FMGMC_OK;
    for (int64_t s0 = 0; s0 < n_samples && rc == FMGMC_OK; s0 += chunk) {
        const int S = int(std::min<int64_t>(chunk, n_samples - s0));
        const double *x = xi + size_t(s0) * M;
        if (!xi_dev) {
            if (hipMemcpyAsync(ctx->main.xi, x, size_t(S) * M * sizeof(double), hipMemcpyHostToDevice, st) !=
                hipSuccess) {
                rc = FMGMC_EHIP;
                break;
            }
            x = ctx->main.xi;
        }
        KLArgs a{};
        a.n = n;
        a.M = M;
        a.xi = x;
        a.phi = ctx->d_phi[level];
        a.kdim = ctx->table.kmax + 1;
        a.ma = ctx->d_ma;
        a.mb = ctx->d_mb;
        a.sqrtlam = ctx->d_sqrtlam;
        a.xw = ctx->main.klx;
        a.nlev = 1;
        a.K64[0] = k_dev ? k_out + size_t(s0) * n * n : tmp;
        rc = launch_kl(a, S, ctx->opts.kl_prec, st);
        if (rc == FMGMC_OK && !k_dev) {
            if (hipMemcpyAsync(k_out + size_t(s0) * n * n, tmp, size_t(S) * n * n * sizeof(double),
                               hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = FMGMC_EHIP;
        }
    }
    if (!xi_dev || !k_dev) (void)hipStreamSynchronize(st);
    dfree(tmp);
    if (rc == FMGMC_EHIP) set_error("fmgmc_synthesize_field: HIP error");
    return rc;
}

int fmgmc_solve_level(fmgmc_ctx *ctx, int32_t level, int64_t n_samples, const double *xi, double *q_fine,
                      double *q_coarse, int32_t *cycles, uint8_t *flags, void *stream) {
    if (!ctx || level < 0 || level >= ctx->hier.n_levels || n_samples < 0 ||
        (n_samples > 0 && (!xi || !q_fine || !q_coarse))) {
        set_error("fmgmc_solve_level: bad arguments");
        return FMGMC_EINVAL;
    }
    DevGuard g(ctx->device);
    bool nc = false, nf = false;
    TRY(solve_level_on(ctx, ctx->main, ctx->tune[level], level, n_samples, xi, q_fine, q_coarse, cycles, flags,
                       reinterpret_cast<hipStream_t>(stream), &nc, &nf));
    return status_of(nc, nf, "fmgmc_solve_level");
}

int fmgmc_solve_levels(fmgmc_ctx *ctx, int32_t n_lev, const int64_t *n_samples, const double *const *xi,
                       double *const *q_fine, double *const *q_coarse, int32_t *const *cycles,
                       uint8_t *const *flags, void *stream) {
    if (!ctx || n_lev < 1 || n_lev > ctx->hier.n_levels || !n_samples || !xi || !q_fine || !q_coarse) {
        set_error("fmgmc_solve_levels: bad arguments");
        return FMGMC_EINVAL;
    }
    for (int l = 0; l < n_lev; ++l)
        if (n_samples[l] < 0 || (n_samples[l] > 0 && (!xi[l] || !q_fine[l] || !q_coarse[l]))) {
            set_error("fmgmc_solve_levels: bad level arguments");
            return FMGMC_EINVAL;
        }
    DevGuard g(ctx->device);
    // the levels' inputs may have been produced on the caller's stream
    FMGMC_HIP(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
    std::vector<Work *> ws(n_lev, nullptr);
    for (int l = 0; l < n_lev; ++l)
        if (n_samples[l] > 0) TRY(level_work(ctx, l, &ws[l]));
    std::vector<int> rcs(n_lev, FMGMC_OK);
    std::vector<std::string> msgs(n_lev);
    std::vector<char> ncs(n_lev, 0), nfs(n_lev, 0);
    // Lanes: one host thread with one stream per hardware queue, so that every
    // lane keeps a hardware queue of its own (the runtime maps streams onto a
    // few hardware queues; two levels sharing one would interleave their many
    // launches in order). Levels go to lanes longest first, each to the lane
    // with the least estimated work (samples x cells, with a floor on the cells
    // for the per-sample cost of the small grids); a lane runs its levels one
    // after another, the first lane on the calling thread.
    std::vector<int> order;
    for (int l = 0; l < n_lev; ++l)
        if (n_samples[l] > 0) order.push_back(l);
    auto cost = [&](int l) {
        const double n = double(ctx->hier.n0 << l);
        return double(n_samples[l]) * std::max(n * n, 4096.0);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    // as many lanes as the runtime has hardware queues (GPU_MAX_HW_QUEUES, 4 by default)
    int hwq = 4;
    if (const char *e = std::getenv("GPU_MAX_HW_QUEUES")) hwq = std::max(1, std::atoi(e));
    const int nl = std::min({int(order.size()), hwq, kMaxLanes});
    while (int(ctx->lanes.size()) < nl) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            set_error("fmgmc_solve_levels: hipStreamCreate failed");
            return FMGMC_EHIP;
        }
        ctx->lanes.push_back(st);
    }
    std::vector<std::vector<int>> lane_levels(nl);
    std::vector<double> load(nl, 0.0);
    for (int l : order) {
        const int j = int(std::min_element(load.begin(), load.end()) - load.begin());
        lane_levels[j].push_back(l);
        load[j] += cost(l);
    }
    auto run_lane = [&](int j) {
        for (int l : lane_levels[j]) {
            (void)hipSetDevice(ctx->device);
            bool nc = false, nf = false;
            rcs[l] = solve_level_on(ctx, *ws[l], ctx->tune[l], l, n_samples[l], xi[l], q_fine[l], q_coarse[l],
                                    cycles ? cycles[l] : nullptr, flags ? flags[l] : nullptr, ctx->lanes[j], &nc,
                                    &nf);
            if (rcs[l] != FMGMC_OK) msgs[l] = g_err;
            ncs[l] = nc;
            nfs[l] = nf;
        }
    };
    std::vector<std::thread> th;
    for (int j = 1; j < nl; ++j) th.emplace_back(run_lane, j);
    if (nl > 0) run_lane(0);
    for (auto &t : th) t.join();
    bool nc = false, nf = false;
    for (int l = 0; l < n_lev; ++l) {
        if (rcs[l] != FMGMC_OK) {
            set_error("fmgmc_solve_levels: level " + std::to_string(l) + ": " + msgs[l]);
            return rcs[l];
        }
        nc |= ncs[l] != 0;
        nf |= nfs[l] != 0;
    }
    return status_of(nc, nf, "fmgmc_solve_levels");
}

int fmgmc_autotune(fmgmc_ctx *ctx, int32_t level, int64_t n_pilot, const double *xi, int32_t *params) {
    if (!ctx || level < 0 || level >= ctx->hier.n_levels || n_pilot < 1 || !xi) {
        set_error("fmgmc_autotune: bad arguments");
        return FMGMC_EINVAL;
    }
    DevGuard g(ctx->device);
    Work *W = nullptr;
    TRY(level_work(ctx, level, &W));
    const int64_t np = std::min<int64_t>(n_pilot, W->S_max);
    double *qf = nullptr, *qc = nullptr, *dxi = nullptr;
    int rc = dalloc(&qf, np);
    if (rc == FMGMC_OK) rc = dalloc(&qc, np);
    if (rc == FMGMC_OK) rc = dalloc(&dxi, size_t(np) * ctx->table.M);
    if (rc == FMGMC_OK &&
        hipMemcpy(dxi, xi, size_t(np) * ctx->table.M * sizeof(double), hipMemcpyDefault) != hipSuccess) {
        set_error("fmgmc_autotune: copy failed");
        rc = FMGMC_EHIP;
    }
    Tune best = ctx->tune[level];
    double best_ms = 1e300;
    const bool saved_prof = ctx->prof;
    ctx->prof = false;
    const int batches[3] = {W->S_max, std::max(1, W->S_max / 2), std::max(1, W->S_max / 4)};
    for (int G : {1, 2, 4, 8}) {
        for (int graphs : {0, 1}) {
            for (int bi = 0; bi < 3 && rc == FMGMC_OK; ++bi) {
                if (bi > 0 && batches[bi] >= np) continue;
                Tune tn;
                tn.check_every = G;
                tn.graphs = graphs;
                tn.batch = batches[bi];
                double ms = 1e300;
                for (int rep = 0; rep < 2 && rc == FMGMC_OK; ++rep) {  // first run warms graphs and caches
                    bool nc = false, nf = false;
                    const auto t0 = std::chrono::steady_clock::now();
                    rc = solve_level_on(ctx, *W, tn, level, np, dxi, qf, qc, nullptr, nullptr, W->own_stream, &nc,
                                        &nf);
                    const auto t1 = std::chrono::steady_clock::now();
                    ms = std::min(ms, std::chrono::duration<double, std::milli>(t1 - t0).count());
                }
                if (rc == FMGMC_OK && ms < best_ms) {
                    best_ms = ms;
                    best = tn;
                }
            }
        }
    }
    ctx->prof = saved_prof;
    dfree(qf);
    dfree(qc);
    dfree(dxi);
    if (rc != FMGMC_OK) return rc;
    ctx->tune[level] = best;
    if (params) {
        params[0] = best.check_every;
        params[1] = best.graphs;
        params[2] = best.batch;
    }
    return write_tune_cache(ctx);
}

int fmgmc_set_schedule(fmgmc_ctx *ctx, int32_t level, const int32_t *params) {
    if (!ctx || level < 0 || level >= ctx->hier.n_levels || !params || params[0] < 1 || params[1] < 0 ||
        params[1] > 1 || params[2] < 0) {
        set_error("fmgmc_set_schedule: bad arguments");
        return FMGMC_EINVAL;
    }
    ctx->tune[level].check_every = params[0];
    ctx->tune[level].graphs = params[1];
    ctx->tune[level].batch = params[2];
    return FMGMC_OK;
}

int fmgmc_get_schedule(const fmgmc_ctx *ctx, int32_t level, int32_t *params) {
    if (!ctx || level < 0 || level >= ctx->hier.n_levels || !params) {
        set_error("fmgmc_get_schedule: bad arguments");
        return FMGMC_EINVAL;
    }
    params[0] = ctx->tune[level].check_every;
    params[1] = ctx->tune[level].graphs;
    params[2] = ctx->tune[level].batch;
    return FMGMC_OK;
}

int fmgmc_set_warm_start(fmgmc_ctx *ctx, const fmgmc_cnn *cnn, int32_t min_n) {
    return fmgmc_set_warm_range(ctx, cnn, min_n, 0);
}

int fmgmc_set_warm_range(fmgmc_ctx *ctx, const fmgmc_cnn *cnn, int32_t min_n, int32_t max_n) {
    if (!ctx || min_n < 16 || max_n < 0 || (cnn && !ir_mode(ctx)) || (cnn && cnn->device != ctx->device) ||
        (cnn && ctx->hier.boundary != FMGMC_BC_MIXED)) {
        set_error("fmgmc_set_warm_start: bad arguments (FP32_IR solver, Case II boundaries, min_n >= 16, same device)");
        return FMGMC_EINVAL;
    }
    DevGuard g(ctx->device);
    if (cnn) {
        TRY(cnn_ensure_packed(const_cast<fmgmc_cnn *>(cnn), nullptr));
        FMGMC_HIP(hipStreamSynchronize(nullptr));
    }
    ctx->warm = cnn;
    ctx->warm_min_n = min_n;
    ctx->warm_max_n = max_n;
    return FMGMC_OK;
}

int fmgmc_cnn_make_data(fmgmc_ctx *ctx, int32_t level, int64_t n_samples, const double *xi, float *x_coarse,
                        float *t_coarse, float *x_fine, float *t_fine, void *stream) {
    if (!ctx || level < 0 || level >= ctx->hier.n_levels || n_samples < 1 || !xi || !x_fine || !t_fine ||
        !ir_mode(ctx) || (!x_coarse) != (!t_coarse) || ctx->hier.boundary != FMGMC_BC_MIXED) {
        set_error("fmgmc_cnn_make_data: bad arguments (FP32_IR solver, Case II boundaries)");
        return FMGMC_EINVAL;
    }
    const int n = ctx->hier.n0 << level;
    if (n < 16 || (x_coarse && (level < 1 || n / 2 < 16))) {
        set_error("fmgmc_cnn_make_data: stage grids must be at least 16 x 16");
        return FMGMC_EINVAL;
    }
    DevGuard g(ctx->device);
    Work &W = ctx->main;
    const size_t need = size_t(W.S_max) * n * n;
    if (W.p0_cap < need) {
        dfree(W.p0);
        W.p0_cap = 0;
        TRY(dalloc(&W.p0, need));
        W.p0_cap = need;
    }
    std::vector<double> qf(n_samples), qc(n_samples);
    W.capx_base[1] = x_fine;
    W.capt_base[1] = t_fine;
    W.capx_base[0] = x_coarse;
    W.capt_base[0] = t_coarse;
    const fmgmc_cnn *warm = ctx->warm;
    ctx->warm = nullptr;  // targets are relative to the plain FMG start
    bool nc = false, nf = false;
    const int rc = solve_level_on(ctx, W, ctx->tune[level], level, n_samples, xi, qf.data(), qc.data(), nullptr,
                                  nullptr, reinterpret_cast<hipStream_t>(stream), &nc, &nf);
    ctx->warm = warm;
    for (int k = 0; k < 2; ++k) W.capx_base[k] = W.capt_base[k] = W.cap_x[k] = W.cap_t[k] = nullptr;
    TRY(rc);
    return status_of(nc, nf, "fmgmc_cnn_make_data");
}

int fmgmc_cnn_train(fmgmc_ctx *ctx, fmgmc_cnn *cnn, int32_t level, int64_t n_samples, const double *xi,
                    int32_t batch, double lr, double *loss_hist) {
    if (!ctx || !cnn || level < 0 || level >= ctx->hier.n_levels || n_samples < 1 || !xi || batch < 1 ||
        !(lr > 0) || cnn->device != ctx->device || ctx->hier.boundary != FMGMC_BC_MIXED) {
        set_error("fmgmc_cnn_train: bad arguments (the network's residual loss is Case II's operator)");
        return FMGMC_EINVAL;
    }
    DevGuard g(ctx->device);
    const int n = ctx->hier.n0 << level, nc = n / 2, M = ctx->table.M;
    const bool coarse = level >= 1 && nc >= 16;
    const int B = int(std::min<int64_t>(batch, std::min<int64_t>(n_samples, ctx->main.S_max)));
    float *xf = nullptr, *tf = nullptr, *xc = nullptr, *tc = nullptr;
    int rc = dalloc(&xf, size_t(B) * 2 * n * n);
    if (rc == FMGMC_OK) rc = dalloc(&tf, size_t(B) * n * n);
    if (rc == FMGMC_OK && coarse) rc = dalloc(&xc, size_t(B) * 2 * nc * nc);
    if (rc == FMGMC_OK && coarse) rc = dalloc(&tc, size_t(B) * nc * nc);
    int64_t h = 0;
    for (int64_t b0 = 0; b0 < n_samples && (rc == FMGMC_OK || rc == FMGMC_ENOTCONV); b0 += B) {
        const int S = int(std::min<int64_t>(B, n_samples - b0));
        rc = fmgmc_cnn_make_data(ctx, level, S, xi + size_t(b0) * M, xc, tc, xf, tf, nullptr);
        if (rc != FMGMC_OK && rc != FMGMC_ENOTCONV) break;
        double loss = 0.0;
        if ((rc = cnn_grad_impl(cnn, n, S, xf, tf, FMGMC_CNN_LOSS_RESIDUAL, &loss, nullptr)) != FMGMC_OK) break;
        if ((rc = cnn_adam_impl(cnn, lr, nullptr)) != FMGMC_OK) break;
        if (loss_hist) loss_hist[h++] = loss;
        if (coarse) {
            if ((rc = cnn_grad_impl(cnn, nc, S, xc, tc, FMGMC_CNN_LOSS_RESIDUAL, &loss, nullptr)) != FMGMC_OK)
                break;
            if ((rc = cnn_adam_impl(cnn, lr, nullptr)) != FMGMC_OK) break;
            if (loss_hist) loss_hist[h++] = loss;
        }
    }
    (void)hipStreamSynchronize(nullptr);
    dfree(xf);
    dfree(tf);
    dfree(xc);
    dfree(tc);
    return rc == FMGMC_ENOTCONV ? FMGMC_OK : rc;
}

int fmgmc_estimate(int32_t n_lev, const int64_t *n, const double *const *qf, const double *const *qc,
                   int32_t n_shifts, fmgmc_est *out) {
    if (!out || n_lev < 1 || n_lev > FMGMC_MAX_LEVELS) {
        set_error("fmgmc_estimate: bad arguments (out NULL or n_lev outside 1..FMGMC_MAX_LEVELS)");
        return FMGMC_EINVAL;
    }
    fmgmc_est e{};
    e.n_levels = n_lev;
    TRY(fmgmc_estimate_levels(n_lev, n, qf, qc, n_shifts, e.level, &e.mean, &e.var_of_mean, nullptr));
    *out = e;
    return FMGMC_OK;
}

int fmgmc_estimate_levels(int32_t n_lev, const int64_t *n, const double *const *qf, const double *const *qc,
                          int32_t n_shifts, fmgmc_level_est *levels, double *mean, double *var_of_mean,
                          void *stream) {
    if (n_lev < 1 || !n || !qf || !qc || n_shifts < 1 || n_shifts > kEstMaxShifts) {
        set_error("fmgmc_estimate: bad arguments");
        return FMGMC_EINVAL;
    }
    for (int l = 0; l < n_lev; ++l)
        if (n[l] < 1 || !qf[l] || !qc[l] || (n_shifts > 1 && (n[l] % n_shifts) != 0)) {
            set_error("fmgmc_estimate: bad level sizes");
            return FMGMC_EINVAL;
        }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *dout = nullptr, *dscr = nullptr;
    int rc = dalloc(&dout, 5);
    if (rc == FMGMC_OK) rc = dalloc(&dscr, kEstMaxShifts);
    EstAcc acc;
    for (int l = 0; l < n_lev && rc == FMGMC_OK; ++l) {
        const double *f = qf[l], *cc = qc[l];
        double *tf = nullptr, *tc = nullptr;
        if (!is_device_ptr(f)) {
            if ((rc = dalloc(&tf, n[l])) != FMGMC_OK) break;
            (void)hipMemcpyAsync(tf, f, n[l] * sizeof(double), hipMemcpyHostToDevice, st);
            f = tf;
        }
        if (!is_device_ptr(cc)) {
            if ((rc = dalloc(&tc, n[l])) != FMGMC_OK) {
                dfree(tf);
                break;
            }
            (void)hipMemcpyAsync(tc, cc, n[l] * sizeof(double), hipMemcpyHostToDevice, st);
            cc = tc;
        }
        rc = launch_level_reduce(f, cc, n[l], n_shifts, dout, dscr, st);
        double h[5] = {0, 0, 0, 0, 0};
        if (rc == FMGMC_OK) {
            if (hipMemcpyAsync(h, dout, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                set_error("fmgmc_estimate: HIP error");
                rc = FMGMC_EHIP;
            }
        }
        dfree(tf);
        dfree(tc);
        if (rc != FMGMC_OK) break;
        acc.add(l, n[l], n_shifts, h, levels);
    }
    dfree(dout);
    dfree(dscr);
    if (rc != FMGMC_OK) return rc;
    acc.finish(mean, var_of_mean);
    return FMGMC_OK;
}

int fmgmc_estimate_levels_noalloc(int32_t n_lev, const int64_t *n, const double *const *qf,
                                  const double *const *qc, int32_t n_shifts, fmgmc_level_est *levels,
                                  double *mean, double *var_of_mean, void *stream) {
    if (n_lev < 1 || !n || !qf || !qc || n_shifts < 1 || n_shifts > kEstMaxShifts) {
        set_error("fmgmc_estimate_levels_noalloc: bad arguments (n_shifts must be 1.." +
                  std::to_string(kEstMaxShifts) + ")");
        return FMGMC_EINVAL;
    }
    for (int l = 0; l < n_lev; ++l) {
        if (n[l] < 1 || !qf[l] || !qc[l] || (n_shifts > 1 && (n[l] % n_shifts) != 0)) {
            set_error("fmgmc_estimate_levels_noalloc: bad level sizes");
            return FMGMC_EINVAL;
        }
        if (!is_device_ptr(qf[l]) || !is_device_ptr(qc[l])) {
            set_error("fmgmc_estimate_levels_noalloc: qf and qc must be device arrays (host arrays would need "
                      "a staging allocation)");
            return FMGMC_EINVAL;
        }
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *scr = nullptr;
    TRY(estimate_scratch(&scr));
    EstAcc acc;
    for (int l = 0; l < n_lev; ++l) {
        TRY(launch_level_reduce(qf[l], qc[l], n[l], n_shifts, scr, scr + kEstShiftOffset, st));
        double h[5] = {0, 0, 0, 0, 0};
        FMGMC_HIP(hipMemcpyAsync(h, scr, sizeof(h), hipMemcpyDeviceToHost, st));
        FMGMC_HIP(hipStreamSynchronize(st));
        acc.add(l, n[l], n_shifts, h, levels);
    }
    acc.finish(mean, var_of_mean);
    return FMGMC_OK;
}

}  // extern "C"
