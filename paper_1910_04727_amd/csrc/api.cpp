// C ABI of the library and the host-side schedule of the full multigrid pass.
//
// Per MLMC level l (Algorithm 3 of the paper), for a device-resident batch of
// samples:
//   1. KL synthesis (matrix cores) -> injected coefficient pyramid;
//   2. correction-operator pyramids (face averaging) for the two QoI stages
//      and the Cholesky factors of the coarsest operators;
//   3. full multigrid: direct solve on the coarsest grid, then for each finer
//      grid an interpolated start and V(nu1,nu2) cycles - one per
//      intermediate stage, and until ||b - A p|| <= tol ||b|| on the stages
//      n_l/2 (gives Q^c_l) and n_l (gives Q^f_l). Converged samples drop out
//      of every later launch through a per-sample activity mask.
//   FP32_IR: cycles in FP32; on the QoI stages FP64 iterative refinement
//   (p64 += e32, r = b - A64 p64) decides convergence and yields the QoI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "common.h"

namespace fmgmc {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

namespace {

constexpr int kMaxGrid = 8;   // grid indices 0..7: 4 .. 512 (n_coarsest = 4) or up to 1024
constexpr int kSmallTop = 32; // grids up to this size run whole cycles in LDS

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

}  // namespace
}  // namespace fmgmc

using namespace fmgmc;

struct fmgmc_ctx {
    fmgmc_field field;
    fmgmc_hier hier;
    fmgmc_opts opts;
    int device = 0;
    ModeTable table;
    int S_max = 0;
    int ng = 0;   // grid levels of the finest MLMC level (indices 0..ng-1)
    int nsz[kMaxGrid] = {};
    int small_top = 0;  // largest grid index handled by the LDS kernel

    // constants
    std::vector<double *> d_phi;  // per MLMC level [kmax+1][n_l]
    int32_t *d_ma = nullptr, *d_mb = nullptr;
    double *d_sqrtlam = nullptr;

    // batch buffers (index = grid level)
    double *K64[kMaxGrid] = {};
    float *K32[kMaxGrid] = {};
    double *x64[kMaxGrid] = {}, *b64[kMaxGrid] = {}, *p64[kMaxGrid] = {};
    float *x32[kMaxGrid] = {}, *b32[kMaxGrid] = {};
    Pyr<double> pf64[2];
    Pyr<float> pf32[2];
    double *chol = nullptr;  // [3][S][N0*N0]: stage operator, coarse-stage pyramid, fine-stage pyramid
    double *rr = nullptr, *q = nullptr, *bnorm = nullptr, *qf = nullptr, *qc = nullptr, *xi = nullptr;
    int32_t *active = nullptr, *cycles = nullptr, *n_active = nullptr;
    uint8_t *flags = nullptr;
    int32_t *h_n_active = nullptr;  // pinned
    double *red_scratch = nullptr;
    // measurement hooks
    struct Rec {
        hipEvent_t a, b;
        double alg;
    };
    bool prof = false;
    std::vector<Rec> prof_rec[FMGMC_PROF_KINDS];
    int top_grid = -1;   // grid index of the finest grid of the solve in progress
    int n_active_host = 0;
};

namespace {

bool ir_mode(const fmgmc_ctx *c) { return c->opts.solver == FMGMC_SOLVER_FP32_IR; }

void free_all(fmgmc_ctx *c) {
    for (auto &p : c->d_phi) dfree(p);
    c->d_phi.clear();
    dfree(c->d_ma); dfree(c->d_mb); dfree(c->d_sqrtlam);
    for (int k = 0; k < kMaxGrid; ++k) {
        dfree(c->K64[k]); dfree(c->K32[k]); dfree(c->x64[k]); dfree(c->b64[k]); dfree(c->p64[k]);
        dfree(c->x32[k]); dfree(c->b32[k]);
        for (int q = 0; q < 2; ++q) {
            dfree(c->pf64[q].f[k].fx); dfree(c->pf64[q].f[k].fy); dfree(c->pf64[q].f[k].fxe);
            dfree(c->pf32[q].f[k].fx); dfree(c->pf32[q].f[k].fy); dfree(c->pf32[q].f[k].fxe);
        }
    }
    dfree(c->chol); dfree(c->rr); dfree(c->q); dfree(c->bnorm); dfree(c->qf); dfree(c->qc); dfree(c->xi);
    dfree(c->active); dfree(c->cycles); dfree(c->n_active); dfree(c->flags); dfree(c->red_scratch);
    if (c->h_n_active) (void)hipHostFree(c->h_n_active);
    c->h_n_active = nullptr;
}

#define TRY(x)                          \
    do {                                \
        int rc_ = (x);                  \
        if (rc_ != FMGMC_OK) return rc_; \
    } while (0)

template <typename T>
int alloc_faces(Faces<T> &f, int S, int n) {
    TRY(dalloc(&f.fx, size_t(S) * n * n));
    TRY(dalloc(&f.fy, size_t(S) * n * n));
    TRY(dalloc(&f.fxe, size_t(S) * n));
    return FMGMC_OK;
}

int allocate(fmgmc_ctx *c) {
    const int S = c->S_max, M = c->table.M;
    const int t = c->ng - 1;
    const bool ir = ir_mode(c);
    for (int k = 0; k <= t; ++k) {
        const size_t N = size_t(S) * c->nsz[k] * c->nsz[k];
        if (!ir) {
            TRY(dalloc(&c->K64[k], N));
            TRY(dalloc(&c->x64[k], N));
            TRY(dalloc(&c->b64[k], N));
        } else {
            TRY(dalloc(&c->K32[k], N));
            TRY(dalloc(&c->x32[k], N));
            TRY(dalloc(&c->b32[k], N));
            // FP64 operator and iterate only where a QoI stage can sit
            if (k >= 1) {
                TRY(dalloc(&c->K64[k], N));
                TRY(dalloc(&c->p64[k], N));
            }
        }
        if (k < t) {
            for (int q = 0; q < 2; ++q) {
                if (q == 0 && k >= t - 1) continue;  // coarse-stage pyramid stops below n_l / 2
                if (!ir) TRY(alloc_faces(c->pf64[q].f[k], S, c->nsz[k]));
                else TRY(alloc_faces(c->pf32[q].f[k], S, c->nsz[k]));
            }
        }
    }
    const int N0 = c->nsz[0] * c->nsz[0];
    TRY(dalloc(&c->chol, size_t(3) * S * N0 * N0));
    TRY(dalloc(&c->rr, S)); TRY(dalloc(&c->q, S)); TRY(dalloc(&c->bnorm, S));
    TRY(dalloc(&c->qf, S)); TRY(dalloc(&c->qc, S)); TRY(dalloc(&c->xi, size_t(S) * M));
    TRY(dalloc(&c->active, S)); TRY(dalloc(&c->cycles, 2 * size_t(S))); TRY(dalloc(&c->n_active, 1));
    TRY(dalloc(&c->flags, S));
    TRY(dalloc(&c->red_scratch, 4096));
    if (hipHostMalloc(reinterpret_cast<void **>(&c->h_n_active), sizeof(int32_t)) != hipSuccess) {
        set_error("hipHostMalloc failed");
        return FMGMC_ENOMEM;
    }
    // tables
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

// ------------------------------------------------------------ measurement
// Brackets one launch with events when profiling is on.
template <typename F>
int timed(fmgmc_ctx *c, int kind, double alg, hipStream_t st, F &&launch) {
    if (!c->prof) return launch();
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

Bufs<double> bufs64(fmgmc_ctx *c) { return {c->K64, c->x64, c->b64, c->pf64}; }
Bufs<float> bufs32(fmgmc_ctx *c) { return {c->K32, c->x32, c->b32, c->pf32}; }

// One cycle with top grid k: top operator from K (stage operator), the levels
// below from correction pyramid q; V(nu1,nu2) on grids above w_max_n, two
// coarse cycles (W) on grids n <= w_max_n. rhs_array: top rhs in b[k] (else the
// Dirichlet data). init: INIT_ZERO / INIT_LOAD / INIT_INTERP (from x[k-1]).
template <typename T>
int vcycle(fmgmc_ctx *c, Bufs<T> B, int S, int k, int q, int init, bool rhs_array, int out_top,
           hipStream_t st) {
    const int nh1 = 2 * c->opts.nu1, nh2 = 2 * c->opts.nu2;
    const int N0 = c->nsz[0] * c->nsz[0];
    const double pW = c->hier.p_west, pE = c->hier.p_east;
    const double *chol_pyr = c->chol + size_t(1 + q) * S * N0 * N0;
    const double *chol_stage = c->chol;
    auto gamma = [&](int j) { return (j > 0 && c->nsz[j] <= c->opts.w_max_n) ? 2 : 1; };
    auto small = [&](int top, bool from_k, int sinit, bool srhs, int sout, const double *chol) {
        SmallArgs<T> a{};
        a.top = top;
        for (int j = 0; j <= top; ++j) a.ns[j] = c->nsz[j];
        a.top_from_k = from_k;
        a.Ktop = B.K[top];
        for (int j = 0; j < kMaxGrid; ++j) a.f[j] = B.pf[q].f[j];
        a.chol = chol;
        a.x = B.x[top];
        a.b = B.b[top];
        a.xc = top > 0 ? B.x[top - 1] : nullptr;
        a.rr = c->rr;
        a.q = c->q;
        a.active = c->active;
        a.pW = pW;
        a.pE = pE;
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
        a.n = c->nsz[j];
        a.x = B.x[j];
        a.b = B.b[j];
        a.K = B.K[j];
        a.f = B.pf[q].f[j];
        a.xc = B.x[j - 1];
        a.bc = B.b[j - 1];
        a.rr = c->rr;
        a.q = c->q;
        a.active = c->active;
        a.pW = pW;
        a.pE = pE;
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
    const double w = sizeof(T), cells = double(c->nsz[k]) * c->nsz[k];
    const bool top = (k == c->top_grid);
    const double act = double(c->n_active_host);
    const double b_pre = (init == INIT_ZERO ? 0.0 : (init == INIT_INTERP ? 0.25 * w : w)) + w /*K*/ +
                         (rhs_array ? w : 0.0) + w /*x out*/ + 0.25 * w /*restricted residual*/;
    const double b_post = w + 0.25 * w + w + (rhs_array ? w : 0.0) + w;
    if (top) TRY(timed(c, FMGMC_PROF_PRE, act * cells * b_pre, st, [&] { return march(k, true, init, rhs_array, OUT_RESTRICT, nh1); }));
    else TRY(march(k, true, init, rhs_array, OUT_RESTRICT, nh1));
    for (int g = 0; g < gamma(k - 1); ++g) TRY(corr(k - 1, g == 0 ? INIT_ZERO : INIT_LOAD));
    if (top) TRY(timed(c, FMGMC_PROF_POST, act * cells * b_post, st, [&] { return march(k, true, INIT_PROLONG, rhs_array, out_top, nh2); }));
    else TRY(march(k, true, INIT_PROLONG, rhs_array, out_top, nh2));
    return FMGMC_OK;
}

int read_active(fmgmc_ctx *c, hipStream_t st, int *out) {
    FMGMC_HIP(hipMemcpyAsync(c->h_n_active, c->n_active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FMGMC_HIP(hipStreamSynchronize(st));
    *out = *c->h_n_active;
    c->n_active_host = *out;
    return FMGMC_OK;
}

int check(fmgmc_ctx *c, int S, int slot, double *qout, int inc, double tol, hipStream_t st, int *n_active) {
    CheckArgs a{};
    a.rr = c->rr;
    a.bnorm = c->bnorm;
    a.q = c->q;
    a.active = c->active;
    a.cycles = c->cycles;
    a.slot = slot;
    a.inc = inc;
    a.flags = c->flags;
    a.qout = qout;
    a.tol = tol;
    a.max_cycles = c->opts.max_cycles;
    a.n_active = c->n_active;
    TRY(launch_check(a, S, st));
    return read_active(c, st, n_active);
}

// Build pyramids and coarsest factors for a batch.
template <typename T>
int prepare(fmgmc_ctx *c, Bufs<T> B, int S, int level, int t, hipStream_t st) {
    const int N0 = c->nsz[0] * c->nsz[0];
    Faces<T> none{};
    TRY(launch_chol<T>(c->nsz[0], B.K[0], none, true, c->chol, S, st));
    for (int q = 0; q < 2; ++q) {
        const int top = (q == 1) ? t : t - 1;   // QoI stage that owns the pyramid
        if (q == 0 && (level == 0 || top < 1)) continue;
        if (top < 1) continue;
        TRY(launch_faces_from_k<T>(c->nsz[top], B.K[top], B.pf[q].f[top - 1], S, st));
        for (int j = top - 1; j >= 1; --j)
            TRY(launch_faces_coarsen<T>(c->nsz[j], B.pf[q].f[j], B.pf[q].f[j - 1], S, st));
        TRY(launch_chol<T>(c->nsz[0], nullptr, B.pf[q].f[0], false, c->chol + size_t(1 + q) * S * N0 * N0, S, st));
    }
    return FMGMC_OK;
}

int run_batch_fp64(fmgmc_ctx *c, int level, int S, double *qf, double *qc, hipStream_t st) {
    const int t = ilog2((c->hier.n0 << level) / c->nsz[0]);
    Bufs<double> B = bufs64(c);
    TRY(prepare<double>(c, B, S, level, t, st));
    const double tol = c->opts.rel_tol;
    for (int k = 0; k <= t; ++k) {
        const bool fine = (k == t), coarse = (level >= 1 && k == t - 1);
        const int q = (level >= 1 && k <= t - 1) ? 0 : 1;
        TRY(launch_fill_i32(c->active, 1, S, st));
        c->n_active_host = S;
        if (!(fine || coarse)) {
            TRY(vcycle<double>(c, B, S, k, q, k == 0 ? INIT_ZERO : INIT_INTERP, false, 0, st));
            continue;
        }
        double *qout = fine ? qf : qc;
        const int slot = fine ? 1 : 0;
        TRY(launch_bnorm<double>(c->nsz[k], B.K[k], c->hier.p_west, c->hier.p_east, c->bnorm, S, st));
        if (k == 0) {  // direct solve: exact, no cycles
            TRY(vcycle<double>(c, B, S, 0, q, INIT_ZERO, false, OUT_RR | OUT_Q, st));
            int na;
            TRY(check(c, S, slot, qout, 0, INFINITY, st, &na));
            continue;
        }
        for (int cyc = 0; cyc < c->opts.max_cycles; ++cyc) {
            TRY(vcycle<double>(c, B, S, k, q, cyc == 0 ? INIT_INTERP : INIT_LOAD, false, OUT_RR | OUT_Q, st));
            int na;
            TRY(check(c, S, slot, qout, 1, tol, st, &na));
            if (na == 0) break;
        }
    }
    return FMGMC_OK;
}

int run_batch_ir(fmgmc_ctx *c, int level, int S, double *qf, double *qc, hipStream_t st) {
    const int t = ilog2((c->hier.n0 << level) / c->nsz[0]);
    Bufs<float> B = bufs32(c);
    TRY(prepare<float>(c, B, S, level, t, st));
    const double tol = c->opts.rel_tol;
    const double pW = c->hier.p_west, pE = c->hier.p_east;
    for (int k = 0; k <= t; ++k) {
        const bool fine = (k == t), coarse = (level >= 1 && k == t - 1);
        const int q = (level >= 1 && k <= t - 1) ? 0 : 1;
        TRY(launch_fill_i32(c->active, 1, S, st));
        c->n_active_host = S;
        if (!(fine || coarse)) {
            TRY(vcycle<float>(c, B, S, k, q, k == 0 ? INIT_ZERO : INIT_INTERP, false, 0, st));
            continue;
        }
        double *qout = fine ? qf : qc;
        const int slot = fine ? 1 : 0;
        const int n = c->nsz[k];
        // FMG start in FP64
        if (fine && level >= 1)
            TRY(launch_interp64<double>(n, c->p64[k - 1], c->p64[k], c->active, pW, pE, S, st));
        else
            TRY(launch_interp64<float>(n, c->x32[k - 1], c->p64[k], c->active, pW, pE, S, st));
        TRY(launch_bnorm<double>(n, c->K64[k], pW, pE, c->bnorm, S, st));
        IRArgs ia{};
        ia.n = n;
        ia.p = c->p64[k];
        ia.e = nullptr;
        ia.K = c->K64[k];
        ia.r32 = c->b32[k];
        ia.rr = c->rr;
        ia.q = c->q;
        ia.active = c->active;
        ia.pW = pW;
        ia.pE = pE;
        {
            // first residual of the stage: reads p and K, writes r (20 B per cell)
            const double irb0 = double(c->n_active_host) * double(n) * n * (8.0 + 8.0 + 4.0);
            if (k == c->top_grid) TRY(timed(c, FMGMC_PROF_IR, irb0, st, [&] { return launch_ir(ia, S, st); }));
            else TRY(launch_ir(ia, S, st));
        }
        const int inner = std::max(1, c->opts.inner_cycles);
        for (int done = 0; done < c->opts.max_cycles; done += inner) {
            for (int ic = 0; ic < inner; ++ic)
                TRY(vcycle<float>(c, B, S, k, q, ic == 0 ? INIT_ZERO : INIT_LOAD, true, 0, st));
            ia.e = c->x32[k];
            const double irb = double(c->n_active_host) * double(n) * n * (8.0 + 4.0 + 8.0 + 8.0 + 4.0);
            if (k == c->top_grid) TRY(timed(c, FMGMC_PROF_IR, irb, st, [&] { return launch_ir(ia, S, st); }));
            else TRY(launch_ir(ia, S, st));
            int na;
            TRY(check(c, S, slot, qout, inner, tol, st, &na));
            if (na == 0) break;
        }
    }
    return FMGMC_OK;
}

int validate(const fmgmc_field *f, const fmgmc_hier *h, const fmgmc_opts *o) {
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    if (!f || !h || !o) return FMGMC_EINVAL;
    if (f->cov_kind != FMGMC_COV_SEPARABLE_EXP || !(f->sigma2 > 0) || !(f->corr_len > 0) || f->n_modes < 1 ||
        f->n_modes > 4096)
        return FMGMC_EINVAL;
    if (h->n_levels < 1 || !pow2(h->n0) || h->n_coarsest != 4 || h->n0 < h->n_coarsest) return FMGMC_EINVAL;
    const int nf = h->n0 << (h->n_levels - 1);
    if (nf > 1024) return FMGMC_EINVAL;
    if (h->n_levels > 1 && h->n0 < 4) return FMGMC_EINVAL;
    if (o->solver != FMGMC_SOLVER_FP64 && o->solver != FMGMC_SOLVER_FP32_IR) return FMGMC_EINVAL;
    if (o->kl_prec < FMGMC_KL_FP64 || o->kl_prec > FMGMC_KL_BF16) return FMGMC_EINVAL;
    if (o->nu1 < 1 || o->nu1 > 2 || o->nu2 < 1 || o->nu2 > 2 || o->max_cycles < 1 || !(o->rel_tol > 0))
        return FMGMC_EINVAL;
    if (o->solver == FMGMC_SOLVER_FP32_IR && h->n0 < 8) return FMGMC_EINVAL;  // QoI stages need n >= 8
    if (o->max_batch < 0 || o->w_max_n < 0) return FMGMC_EINVAL;
    return FMGMC_OK;
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

}  // namespace

extern "C" {

const char *fmgmc_last_error(void) { return g_err.c_str(); }

int fmgmc_version(void) { return 100; }

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
    c->S_max = opts->max_batch > 0 ? opts->max_batch : 1024;
    int rc = build_mode_table(field->sigma2, field->corr_len, field->n_modes, c->table);
    if (rc != FMGMC_OK) {
        set_error("fmgmc_create: mode table");
        return rc;
    }
    const int nf = hier->n0 << (hier->n_levels - 1);
    c->ng = ilog2(nf / hier->n_coarsest) + 1;
    if (c->ng > kMaxGrid) {
        set_error("fmgmc_create: too many grid levels");
        return FMGMC_EINVAL;
    }
    for (int k = 0; k < c->ng; ++k) c->nsz[k] = hier->n_coarsest << k;
    c->small_top = ilog2(kSmallTop / hier->n_coarsest);
    rc = allocate(c.get());
    if (rc != FMGMC_OK) {
        free_all(c.get());
        return rc;
    }
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
        if (rc == FMGMC_OK && (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess)) {
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
    free_all(ctx);
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

int fmgmc_synthesize_field(fmgmc_ctx *ctx, int32_t level, int64_t n_samples, const double *xi, double *k_out, void *stream) {
    if (!ctx || level < 0 || level >= ctx->hier.n_levels || n_samples < 0 || (n_samples > 0 && (!xi || !k_out))) {
        set_error("fmgmc_synthesize_field: bad arguments");
        return FMGMC_EINVAL;
    }
    DevGuard g(ctx->device);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int n = ctx->hier.n0 << level, M = ctx->table.M;
    const bool xi_dev = is_device_ptr(xi), k_dev = is_device_ptr(k_out);
    double *tmp = nullptr;
    const int chunk = ctx->S_max;
    if (!k_dev) TRY(dalloc(&tmp, size_t(chunk) * n * n));
    int rc = FMGMC_OK;
    for (int64_t s0 = 0; s0 < n_samples && rc == FMGMC_OK; s0 += chunk) {
        const int S = int(std::min<int64_t>(chunk, n_samples - s0));
        const double *x = xi + size_t(s0) * M;
        if (!xi_dev) {
            if (hipMemcpyAsync(ctx->xi, x, size_t(S) * M * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess) {
                rc = FMGMC_EHIP;
                break;
            }
            x = ctx->xi;
        }
        KLArgs a{};
        a.n = n;
        a.M = M;
        a.xi = x;
        a.phi = ctx->d_phi[level];
        a.ma = ctx->d_ma;
        a.mb = ctx->d_mb;
        a.sqrtlam = ctx->d_sqrtlam;
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
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int M = ctx->table.M;
    const int n = ctx->hier.n0 << level;
    const int t = ilog2(n / ctx->nsz[0]);
    const bool ir = ir_mode(ctx);
    const bool xi_dev = is_device_ptr(xi), qf_dev = is_device_ptr(q_fine), qc_dev = is_device_ptr(q_coarse);
    const bool cy_dev = cycles && is_device_ptr(cycles), fl_dev = flags && is_device_ptr(flags);
    bool any_notconv = false, any_nonfinite = false;
    std::vector<uint8_t> hflags;
    for (int64_t s0 = 0; s0 < n_samples; s0 += ctx->S_max) {
        const int S = int(std::min<int64_t>(ctx->S_max, n_samples - s0));
        const double *x = xi + size_t(s0) * M;
        if (!xi_dev) {
            FMGMC_HIP(hipMemcpyAsync(ctx->xi, x, size_t(S) * M * sizeof(double), hipMemcpyHostToDevice, st));
            x = ctx->xi;
        }
        double *qf = qf_dev ? q_fine + s0 : ctx->qf;
        double *qc = qc_dev ? q_coarse + s0 : ctx->qc;
        TRY(launch_fill_i32(ctx->cycles, 0, 2 * int64_t(S), st));
        TRY(launch_fill_u8(ctx->flags, 0, S, st));
        TRY(launch_fill_f64(qc, 0.0, S, st));
        KLArgs a{};
        a.n = n;
        a.M = M;
        a.xi = x;
        a.phi = ctx->d_phi[level];
        a.ma = ctx->d_ma;
        a.mb = ctx->d_mb;
        a.sqrtlam = ctx->d_sqrtlam;
        a.nlev = t + 1;
        for (int j = 0; j <= t; ++j) {
            const int k = t - j;  // pyramid slot j = grid index t - j
            a.K64[j] = ctx->K64[k];
            a.K32[j] = ir ? ctx->K32[k] : nullptr;
            if (ir && !(k == t || (level >= 1 && k == t - 1))) a.K64[j] = nullptr;
        }
        ctx->top_grid = t;
        const double klf = 2.0 * double(M) * double(n) * n * S;
        TRY(timed(ctx, FMGMC_PROF_KL, klf, st, [&] { return launch_kl(a, S, ctx->opts.kl_prec, st); }));
        TRY(ir ? run_batch_ir(ctx, level, S, qf, qc, st) : run_batch_fp64(ctx, level, S, qf, qc, st));
        // outputs
        if (!qf_dev) FMGMC_HIP(hipMemcpyAsync(q_fine + s0, qf, S * sizeof(double), hipMemcpyDeviceToHost, st));
        if (!qc_dev) FMGMC_HIP(hipMemcpyAsync(q_coarse + s0, qc, S * sizeof(double), hipMemcpyDeviceToHost, st));
        if (cycles)
            FMGMC_HIP(hipMemcpyAsync(cycles + 2 * s0, ctx->cycles, 2 * size_t(S) * sizeof(int32_t),
                                     cy_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
        if (flags && fl_dev)
            FMGMC_HIP(hipMemcpyAsync(flags + s0, ctx->flags, S, hipMemcpyDeviceToDevice, st));
        hflags.resize(S);
        FMGMC_HIP(hipMemcpyAsync(hflags.data(), ctx->flags, S, hipMemcpyDeviceToHost, st));
        FMGMC_HIP(hipStreamSynchronize(st));
        if (flags && !fl_dev) std::memcpy(flags + s0, hflags.data(), S);
        for (int s = 0; s < S; ++s) {
            any_notconv |= (hflags[s] & FMGMC_FLAG_NOTCONV) != 0;
            any_nonfinite |= (hflags[s] & FMGMC_FLAG_NONFINITE) != 0;
        }
    }
    if (any_nonfinite) {
        set_error("fmgmc_solve_level: non-finite residual in some samples (see flags)");
        return FMGMC_ENONFINITE;
    }
    if (any_notconv) {
        set_error("fmgmc_solve_level: some samples did not reach rel_tol (see flags)");
        return FMGMC_ENOTCONV;
    }
    return FMGMC_OK;
}

int fmgmc_estimate(int32_t n_lev, const int64_t *n, const double *const *qf, const double *const *qc,
                   int32_t n_shifts, fmgmc_level_est *levels, double *mean, double *var_of_mean, void *stream) {
    if (n_lev < 1 || !n || !qf || !qc || n_shifts < 1 || n_shifts > 4096) {
        set_error("fmgmc_estimate: bad arguments");
        return FMGMC_EINVAL;
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    double *dout = nullptr, *dscr = nullptr;
    TRY(dalloc(&dout, 5));
    TRY(dalloc(&dscr, 4096));
    double total = 0.0, totc = 0.0, var = 0.0;  // compensated over levels
    int rc = FMGMC_OK;
    for (int l = 0; l < n_lev && rc == FMGMC_OK; ++l) {
        if (n[l] < 1 || !qf[l] || !qc[l] || (n_shifts > 1 && (n[l] % n_shifts) != 0)) {
            set_error("fmgmc_estimate: bad level sizes");
            rc = FMGMC_EINVAL;
            break;
        }
        const double *f = qf[l], *cc = qc[l];
        double *tf = nullptr, *tc = nullptr;
        if (!is_device_ptr(f)) {
            if ((rc = dalloc(&tf, n[l])) != FMGMC_OK) break;
            (void)hipMemcpyAsync(tf, f, n[l] * sizeof(double), hipMemcpyHostToDevice, st);
            f = tf;
        }
        if (!is_device_ptr(cc)) {
            if ((rc = dalloc(&tc, n[l])) != FMGMC_OK) { dfree(tf); break; }
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
        if (levels) {
            levels[l].n = n[l];
            levels[l].mean_y = h[0];
            levels[l].var_y = h[1];
            levels[l].mean_qf = h[2];
            levels[l].var_qf = h[3];
            levels[l].mean_qc = h[4];
        }
        // Neumaier over the (few) levels
        const double tt = total + h[0];
        totc += (std::fabs(total) >= std::fabs(h[0])) ? (total - tt) + h[0] : (h[0] - tt) + total;
        total = tt;
        var += (n_shifts > 1) ? h[1] : h[1] / double(n[l]);
    }
    dfree(dout);
    dfree(dscr);
    if (rc != FMGMC_OK) return rc;
    if (mean) *mean = total + totc;
    if (var_of_mean) *var_of_mean = var;
    return FMGMC_OK;
}

}  // extern "C"
