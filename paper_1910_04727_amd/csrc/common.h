// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fmgmc.h"

namespace fmgmc {

void set_error(const std::string &msg);

#define FMGMC_HIP(call)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            ::fmgmc::set_error(std::string(#call) + ": " + hipGetErrorString(e_));            \
            return FMGMC_EHIP;                                                                 \
        }                                                                                      \
    } while (0)

// 1/x on the device: the hardware reciprocal (FP32, within 1 ulp); in FP64
// refined by two Newton steps to full double precision
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// Workgroups are handed to the chip's 8 XCDs in turn (workgroup i to XCD
// i mod 8), each XCD with its own L2. xcd_unit maps workgroup L of T to a work
// unit so that every XCD takes one contiguous range of units: neighbouring
// units (consecutive rows of one sample) that read the same input rows then
// meet in the same L2 instead of fetching them from HBM once per XCD.
__device__ __forceinline__ int xcd_unit(int L, int T) {
    const int q = T >> 3, r = T & 7, x = L & 7;
    return x * q + min(x, r) + (L >> 3);
}

// ---------------------------------------------------------------- KL table
struct ModeTable {
    int M = 0;
    int kmax = 0;                 // largest 1-D index used (0-based)
    std::vector<int32_t> a, b;    // x / y 1-D mode index of 2-D mode m
    std::vector<double> lam;      // sigma^2 theta_a theta_b
    std::vector<double> w;        // 1-D roots w_k, k = 0..kmax
};
int build_mode_table(double sigma2, double corr_len, int M, ModeTable &t);
// phi_k(s) (0-based k) on the points s_i = i / n, i < n: tab[k * n + i]
void tabulate_phi(const ModeTable &t, int n, std::vector<double> &tab);

// ---------------------------------------------------------------- kernels
// Boundary conditions (Table 1): Dirichlet values on the west, east, south and
// north sides. all = 0: Case II (no flow through the south and north sides, QoI
// = outflow through the east side); all = 1: Case I (Dirichlet on every side,
// QoI = pressure at the centre, the mean of the four centre cells).
struct Bnd {
    double w, e, s, n;
    int all;
};

// Per-level views of a batch (S samples, grid n x n, sample stride n*n).
template <typename T>
struct Faces {
    T *fx;    // [S][n][n] west face of each cell (face i of row j)
    T *fy;    // [S][n][n] south face of each cell (face j of column i); row 0 is the
              //           south boundary face (0 in Case II)
    T *fxe;   // [S][n]    east boundary face of each row
    T *fyn;   // [S][n]    north boundary face of each column (0 in Case II)
};

// march kernels: one workgroup per sample marching over the rows
// INIT_IR (FP32, stage operator): zero start; the right-hand side of each row
// is the FP64 refinement residual of the stage iterate p, formed in the same
// pass (with OUT_PUPD, p += e first and p written back), and K = float(K64).
// OUT_FACES (INIT_IR without OUT_PUPD): the pass also writes the correction
// faces on n/2 (f), those that k_faces_from_k forms from K, from its own
// coefficient ring. OUT_PINTERP (with OUT_FACES): p is not read but formed as
// the FMG interpolation of the FP64 solution on n/2 (pc), as k_interp64 forms
// it, and written.
enum { INIT_ZERO = 0, INIT_LOAD = 1, INIT_PROLONG = 2, INIT_INTERP = 3, INIT_IR = 4 };
enum { OUT_RESTRICT = 1, OUT_RR = 2, OUT_Q = 4, OUT_PUPD = 8, OUT_FACES = 16, OUT_PINTERP = 32 };

template <typename T>
struct MarchArgs {
    int n;
    T *x;                 // [S][n][n]
    const T *b;           // [S][n][n] right-hand side (RHS array mode)
    const T *K;           // [S][n][n] stage coefficient (coefficients from K)
    Faces<T> f;           // correction faces (coefficients from faces)
    const T *xc;          // [S][n/2][n/2] coarse correction (PROLONG) or solution (INTERP)
    T *bc;                // [S][n/2][n/2] restricted residual (OUT_RESTRICT)
    double *rr;           // [S] sum of squared residuals (OUT_RR)
    double *q;            // [S] QoI (OUT_Q)
    const int32_t *active;// [S] nonzero = sample still iterating
    Bnd g;
    // INIT_IR only: the refinement's operands (rr and q then take its FP64
    // residual norm and QoI)
    double *p;            // [S][n][n] FP64 stage iterate
    const double *pc;     // [S][n/2][n/2] FP64 solution on n/2 (OUT_PINTERP)
    const float *e;       // [S][n][n] FP32 correction added to p (OUT_PUPD)
    const double *K64;    // [S][n][n] stage coefficient in FP64
    float *r32;           // [S][n][n] the residual, rounded to FP32
};

// Launches one fused smoothing pass; nhalf = number of half-sweeps (2 nu),
// coef_from_k: stage operator from K (else correction faces), rhs_array: b given
// (else Dirichlet data), init / out as above.
template <typename T>
int launch_march(const MarchArgs<T> &a, int S, int nhalf, bool coef_from_k, int init,
                 bool rhs_array, int out, hipStream_t st);

// face pyramid: from the stage operator on n (K) or from faces on n, to faces on n/2
template <typename T>
int launch_faces_from_k(int n, const T *K, int all, Faces<T> out, int S, hipStream_t st);
template <typename T>
int launch_faces_coarsen(int n, Faces<T> in, Faces<T> out, int S, hipStream_t st);

// small grids: a whole V-cycle per workgroup in LDS
template <typename T>
struct SmallArgs {
    int top;              // level index of the cycle's top grid (grid 4 << top... see ns)
    int ns[8];            // grid size of level k (k = 0 coarsest)
    bool top_from_k;      // top operator = stage operator from K (else faces)
    const T *Ktop;        // [S][n_top][n_top]
    Faces<T> f[8];        // correction faces per level (levels below top, and top if !top_from_k)
    const double *chol;   // [S][N0][N0] inverse of the coarsest operator (FP64)
    T *x;                 // [S][n_top^2] in/out
    const T *b;           // [S][n_top^2] rhs (array mode)
    const T *xc;          // interp source [S][(n_top/2)^2] (INIT_INTERP)
    double *rr;
    double *q;
    const int32_t *active;
    Bnd g;
    int nu1, nu2;
    int wmax;             // coarse grids with n <= wmax (not the coarsest) are cycled twice
};
template <typename T>
int launch_small(const SmallArgs<T> &a, int S, int init, bool rhs_array, int out, hipStream_t st);

// Inverse of the coarsest operator (n0 x n0 grid, n0^2 <= 16) from K or faces,
// through its Cholesky factor, in FP64.
template <typename T>
int launch_chol(int n0, const T *K, Faces<T> f, bool from_k, int all, double *L, int S, hipStream_t st);

// KL synthesis: K_top (and its injected pyramid) from xi.
struct KLArgs {
    int n;                // finest grid of the level
    int M;
    const double *xi;     // [S][M]
    const double *phi;    // [kdim][n] 1-D eigenfunctions on the grid points
    int kdim;             // 1-D modes per axis in use (kmax + 1)
    const int32_t *ma, *mb;
    const double *sqrtlam;// [M]
    int nlev;             // pyramid levels written (finest first): n, n/2, ...
    double *K64[9];       // nullable per level
    float *K32[9];        // nullable per level
    void *xw;             // FP32 / BF16 contraction: xi in operand order, kl_work_bytes(S, M, prec) bytes
};
// device bytes of the xi workspace launch_kl needs for S samples (0: none)
size_t kl_work_bytes(int S, int M, int prec);
int launch_kl(const KLArgs &a, int S, int prec, hipStream_t st);
// whether launch_kl takes the separable path, and its flops per sample
bool kl_separable(const KLArgs &a, int prec);
double kl_flops(const KLArgs &a, int prec);

// FP64 refinement: p += e (optional), r = b - A p (FP64, K64 stage operator),
// r -> r32 (rhs of the next inner cycles), rr, Q.
struct IRArgs {
    int n;
    double *p;
    const float *e;       // nullable: no update
    const double *K;
    float *r32;
    double *rr, *q;
    const int32_t *active;
    Bnd g;
};
int launch_ir(const IRArgs &a, int S, hipStream_t st);

// p64 (n) = FMG interpolation of xc (n/2), xc float or double
template <typename TS>
int launch_interp64(int n, const TS *xc, double *p, const int32_t *active, const Bnd &g, int S,
                    hipStream_t st);

// ||b||_2 of the stage right-hand side (Dirichlet data through the boundary faces)
template <typename T>
int launch_bnorm(int n, const T *K, const Bnd &g, double *bn, int S, hipStream_t st);

// convergence bookkeeping for one QoI stage after a cycle
struct CheckArgs {
    const double *rr, *bnorm, *q;
    int32_t *active;
    int32_t *cycles;      // [S][2]
    int slot;             // 0 coarse stage, 1 fine stage
    int inc;              // V-cycles done since the last check (0: direct solve)
    uint8_t *flags;
    double *qout;         // [S]
    double tol;
    int max_cycles;
    int32_t *n_active;    // single int: number still active after the check
};
int launch_check(const CheckArgs &a, int S, hipStream_t st);
int launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);
int launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t st);
int launch_fill_f64(double *p, double v, int64_t n, hipStream_t st);

// estimators: compensated sums in a fixed order
int launch_level_reduce(const double *qf, const double *qc, int64_t n, int nshift, double *out,
                        double *shift_means, hipStream_t st);
// Allocation-free estimator: the per-device address of the library's fixed
// scratch array (kEstScratchDoubles doubles: 5 results at 0, per-shift means
// from kEstShiftOffset, at most kEstMaxShifts of them), looked up on first use.
constexpr int kEstMaxShifts = 4096;
constexpr int kEstShiftOffset = 8;
constexpr int kEstScratchDoubles = kEstShiftOffset + kEstMaxShifts;
constexpr int kMaxDevices = 64;
int estimate_scratch(double **out);

}  // namespace fmgmc
